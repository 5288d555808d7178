"""GPU parity of the batched multi-scene launch (rt_trace_batch): bit-identical
to one rt_trace_closest launch per scene and to oracle B, for every
intersector, with counters; graph capture and replay; the autotuner."""
import numpy as np
import pytest

from paper_1912_12786_amd import workloads as W
from tests import parity as P

pytestmark = pytest.mark.gpu
MISS = 0xFFFFFFFF


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1912_12786_amd import rtx
    rtx.load_library()
    return torch, rtx


def small_batch(n_scenes=12, alpha=False):
    scenes = W.batched(n_scenes, tri_range=(1_000, 20_000), ray_range=(1_000, 20_000))
    if alpha:
        for i, s in enumerate(scenes):
            v, tc, geom = W.billboard_quads(max(1, s["vertices"].shape[0] // 2), 1000 + i,
                                            W.BILLBOARD_EYE, n_tex=4)
            s["vertices"], s["texcoords"], s["geom_ids"] = v, tc, geom
            s["textures"] = W.alpha_textures(4, 64, 2000 + i)
    return scenes


def upload(rtx, scenes):
    return [rtx.upload_scene(s["vertices"], s.get("geom_ids"), s.get("texcoords"),
                             s.get("textures")) for s in scenes]


def per_scene(torch, rtx, sc_list, scenes, kind, count, **kw):
    outs, cnts = [], []
    for sc, s in zip(sc_list, scenes):
        r = torch.from_numpy(s["rays"]).cuda()
        if count:
            h, c = rtx.trace(sc, r, kind, count=True, **kw)
            cnts.append(c)
        else:
            h = rtx.trace(sc, r, kind, **kw)
        outs.append(h)
    torch.cuda.synchronize()
    return torch.cat(outs), (torch.cat(cnts) if count else None)


def same_bits(a, b):
    import torch
    return a.shape == b.shape and torch.equal(a.view(torch.int32), b.view(torch.int32))


@pytest.mark.parametrize("kind", ["default", "alpha", "procedural"])
def test_small_batch_matches_per_scene_and_oracle(env, oracle_lib, kind):
    torch, rtx = env
    scenes = small_batch(alpha=(kind == "alpha"))
    announce(f"small batch {len(scenes)} scenes kind={kind}")
    sc_list = upload(rtx, scenes)
    kw = dict(alpha_min=128) if kind == "alpha" else (dict(checker_n=8) if kind == "procedural" else {})
    batch = rtx.Batch(sc_list, [s["rays"].shape[0] for s in scenes], kind)
    rays = torch.from_numpy(np.concatenate([s["rays"] for s in scenes])).cuda()
    hits, cnt = batch.trace(rays, count=True, **({"checker_n": 8} if kind == "procedural" else {}))
    torch.cuda.synchronize()
    ref_h, ref_c = per_scene(torch, rtx, sc_list, scenes, kind, True, **kw)
    assert same_bits(hits, ref_h) and same_bits(cnt, ref_c)
    g = P.hits_to_numpy(hits)
    c = cnt.cpu().numpy()
    off = batch.offsets
    for i, s in enumerate(scenes):
        okw = {}
        if kind == "alpha":
            okw = dict(geom_ids=s["geom_ids"], texcoords=s["texcoords"], textures=s["textures"],
                       alpha_min=128)
        elif kind == "procedural":
            okw = dict(checker_n=8)
        bvh = oracle_lib.build_bvh(s["vertices"])
        B = oracle_lib.traverse(s["vertices"], bvh, s["rays"], kind, **okw)
        sl = slice(off[i], off[i + 1])
        P.assert_exact_vs_b({k: v[sl] for k, v in g.items()}, B, f"batch scene {i}")
        assert np.array_equal(c[sl].view(np.uint32), B["counters"])
        # and the float64 definition on up to 512 rays of the scene
        rng = np.random.default_rng(100 + i)
        idx = np.sort(rng.choice(s["rays"].shape[0], size=min(512, s["rays"].shape[0]),
                                 replace=False))
        A = oracle_lib.brute(s["vertices"], s["rays"], kind, ray_index=idx, **okw)
        P.compare_vs_a({k: v[sl] for k, v in g.items()}, A, idx, f"batch scene {i} vs A")


def test_full_batch_matches_per_scene_and_oracle(env, oracle_lib):
    """The benchmark's 64-scene batch (5.1 M triangles, 19.9 M rays): one
    batched launch equals 64 per-scene launches bit for bit, every ray of
    every scene equals oracle B (hits and counters), and 512 rays per scene
    match the float64 definition outside its exception set."""
    from concurrent.futures import ThreadPoolExecutor
    torch, rtx = env
    scenes = W.batched()
    announce(f"full batch: {len(scenes)} scenes, {sum(s['vertices'].shape[0] for s in scenes)} "
             f"tris, {sum(s['rays'].shape[0] for s in scenes)} rays")
    sc_list = upload(rtx, scenes)
    batch = rtx.Batch(sc_list, [s["rays"].shape[0] for s in scenes], "default")
    rays = torch.from_numpy(np.concatenate([s["rays"] for s in scenes])).cuda()
    hits, cnt = batch.trace(rays, count=True)
    ref, _ = per_scene(torch, rtx, sc_list, scenes, "default", False)
    assert same_bits(hits, ref)
    g = P.hits_to_numpy(hits)
    c = cnt.cpu().numpy()
    # the oracle's builds are single-threaded: build the 64 BVHs side by side
    with ThreadPoolExecutor(8) as pool:
        bvhs = list(pool.map(lambda s: oracle_lib.build_bvh(s["vertices"]), scenes))
    off = batch.offsets
    checked = excluded = 0
    for i, (s, bvh) in enumerate(zip(scenes, bvhs)):
        sl = slice(off[i], off[i + 1])
        B = oracle_lib.traverse(s["vertices"], bvh, s["rays"], "default")
        P.assert_exact_vs_b({k: v[sl] for k, v in g.items()}, B, f"full batch scene {i}")
        assert np.array_equal(c[sl].view(np.uint32), B["counters"]), f"counters of scene {i}"
        rng = np.random.default_rng(200 + i)
        idx = np.sort(rng.choice(s["rays"].shape[0], size=min(512, s["rays"].shape[0]),
                                 replace=False))
        A = oracle_lib.brute(s["vertices"], s["rays"], "default", ray_index=idx)
        r = P.compare_vs_a({k: v[sl] for k, v in g.items()}, A, idx, f"full batch scene {i} vs A")
        checked += r["checked"]
        excluded += r["excluded"]
    print(f"[gpu-case] full batch vs the float64 definition: {checked} rays checked, "
          f"{excluded} in the exception set", flush=True)
    assert excluded <= 0.01 * (checked + excluded)


def test_batch_graph_capture_replays(env):
    torch, rtx = env
    scenes = small_batch(8)
    announce("batch launch captured in a graph, replayed with eager work between")
    sc_list = upload(rtx, scenes)
    batch = rtx.Batch(sc_list, [s["rays"].shape[0] for s in scenes], "default")
    rays = torch.from_numpy(np.concatenate([s["rays"] for s in scenes])).cuda()
    ws = rtx.Workspace("cuda")
    out = torch.empty((rays.shape[0], 4), device="cuda")
    eager = batch.trace(rays, workspace=ws).clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.trace(rays, out=out, workspace=ws)      # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.trace(rays, out=out, workspace=ws)
    for rep in range(3):
        out.fill_(-1.0)
        per_scene(torch, rtx, sc_list[:2], scenes[:2], "default", False)   # unrelated eager work
        g.replay()
        torch.cuda.synchronize()
        assert same_bits(out, eager), rep


def test_autotuner_picks_a_compiled_shape(env, tmp_path):
    torch, rtx = env
    from paper_1912_12786_amd import autotune
    scenes = small_batch(6)
    announce("autotuner over the small batch")
    sc_list = upload(rtx, scenes)
    batch = rtx.Batch(sc_list, [s["rays"].shape[0] for s in scenes], "default")
    rays = torch.from_numpy(np.concatenate([s["rays"] for s in scenes])).cuda()
    ws = rtx.Workspace("cuda")
    ref = batch.trace(rays, workspace=ws).clone()
    best, times = autotune.tune("small-batch",
                                lambda sh: batch.trace(rays, workspace=ws, shape=sh),
                                cache_path=str(tmp_path / "tune.json"), steps=3, warmup=1)
    assert tuple(best) in {tuple(s) for s in rtx.rt_launch_shapes()}
    assert len(times) == len(rtx.rt_launch_shapes())
    assert same_bits(batch.trace(rays, workspace=ws, shape=best), ref)
    again, _ = autotune.tune("small-batch", lambda sh: None, cache_path=str(tmp_path / "tune.json"))
    assert tuple(again) == tuple(best)      # served from the cache
