"""Performance smoke test: the benchmark's launch (alpha mask, billboards
200k triangles, 1920x1080, leaves of at most 2 triangles packed into 48-byte
nodes, 8x8 tiles, longest path first) must keep at least half of its recorded
throughput (3,527-3,565 Mrays/s on MI355X, 0.58 ms per step).
The bound is loose on purpose: it catches a broken schedule or a lost
optimisation, not run-to-run noise.  The roofline object bench.py builds from
the same launch time must describe a physically possible point: measured HBM
traffic over the launch time at most the 8 TB/s peak, the texture addresser
busy at most all of the time."""
import pytest

from paper_1912_12786_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_headline_throughput_floor():
    import torch
    import bench
    from paper_1912_12786_amd import rtx
    rtx.load_library()
    assert torch.cuda.is_available()
    print("[gpu-case] perf smoke: billboards alpha, 20 timed launches", flush=True)
    wl = W.billboards()
    scene = rtx.upload_scene(wl.vertices, wl.geom_ids, wl.texcoords, wl.textures, max_leaf=2,
                             layout="f32p")
    rays = torch.from_numpy(wl.rays).cuda()
    out = torch.empty((wl.n_rays, 4), dtype=torch.float32, device="cuda")
    ws = rtx.Workspace("cuda")
    stream = torch.cuda.current_stream()
    ms = bench.timed(lambda: rtx.trace(scene, rays, "alpha", alpha_min=128, out=out, workspace=ws,
                                       image_width=1920, longest_first=True), 20, 3, stream)
    mrays = wl.n_rays / ms / 1e3
    rec = bench.find_counters(bench.kernel_source_sha(), wl.name, "alpha", "closest", "f32p", 2,
                              list(rtx.rt_launch_shapes()[0]), "scanline", "tiles",
                              "longest-first", rtx.RT_DEFAULT_WAVES_PER_SIMD)
    roof = bench.roofline(ms, 0, rec)
    print(f"[gpu-case] {mrays:.0f} Mrays/s, {ms:.4f} ms, HBM fraction {roof['frac']}, "
          f"counters {None if rec is None else rec['file']}", flush=True)
    assert mrays > 1760, mrays
    if rec is not None:
        assert 0 < roof["frac"] <= 1.0, roof
        assert 0 < roof["issue"]["frac"] <= 1.0, roof
