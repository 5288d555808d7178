"""Performance smoke test: the benchmark's launch (alpha mask, billboards
200k triangles, 1920x1080, leaves of at most 2 triangles) must keep at least
half of its recorded throughput (3197 Mrays/s, 0.643 ms per launch on MI355X)
and of its algorithmic-bandwidth fraction (1.11 of the 8 TB/s HBM peak).  The
bounds are loose on purpose: they catch a broken schedule or a lost
optimisation, not run-to-run noise."""
import numpy as np
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
    scene = rtx.upload_scene(wl.vertices, wl.geom_ids, wl.texcoords, wl.textures, max_leaf=2)
    rays = torch.from_numpy(wl.rays).cuda()
    out = torch.empty((wl.n_rays, 4), dtype=torch.float32, device="cuda")
    ws = rtx.Workspace("cuda")
    stream = torch.cuda.current_stream()
    ms = bench.timed(lambda: rtx.trace(scene, rays, "alpha", alpha_min=128, out=out, workspace=ws),
                     20, 3, stream)
    mrays = wl.n_rays / ms / 1e3
    _, cnt = rtx.trace(scene, rays, "alpha", alpha_min=128, count=True, workspace=ws)
    torch.cuda.synchronize()
    alg = int(bench.bytes_per_ray(cnt.cpu().numpy().view(np.uint32), "alpha").sum())
    frac = alg / (ms * 1e-3) / (bench.PEAK_HBM_GBS * 1e9)
    print(f"[gpu-case] {mrays:.0f} Mrays/s, {ms:.4f} ms, roofline fraction {frac:.3f}", flush=True)
    assert mrays > 1550, mrays
    assert frac > 0.55, frac
