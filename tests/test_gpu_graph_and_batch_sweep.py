"""Graph capture of the single-scene entry points (closest, any, multi,
instanced), replayed with eager work in between and checked against the eager
results every time; and seeded random batches (random scene sizes and kinds,
per-scene alpha textures and thresholds) against oracle B, bit for bit."""
import numpy as np
import pytest

from paper_1912_12786_amd import workloads as W
from tests import parity as P
from tests.test_gpu_random import random_case
from tests.test_oracle_pins import _scene_params

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1912_12786_amd import rtx
    rtx.load_library()
    return torch, rtx


def same_bits(a, b):
    import torch
    return a.shape == b.shape and torch.equal(a.view(torch.int32), b.view(torch.int32))


@pytest.mark.parametrize("query", ["closest", "any", "multi", "instanced"])
def test_graph_replays_match_eager(env, query):
    torch, rtx = env
    announce(f"graph capture of {query}")
    wl = W.tiny()
    rng = np.random.default_rng(9)
    ai = dict(geom_ids=rng.integers(0, 4, size=wl.n_tris).astype(np.uint32),
              texcoords=rng.uniform(0, 1, size=(wl.n_tris, 3, 2)).astype(np.float32),
              textures=W.alpha_textures(4, 64, 9))
    sc = rtx.upload_scene(wl.vertices, ai["geom_ids"], ai["texcoords"], ai["textures"])
    rays = torch.from_numpy(wl.rays).cuda()
    ws = rtx.Workspace("cuda")
    if query == "instanced":
        maps = np.array([[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0],
                         [1, 0, 0, -0.3, 0, 1, 0, 0, 0, 0, 1, 0]], np.float32)
        from tests.test_oracle_instances import world_boxes
        lo, hi = world_boxes(wl.vertices, maps)
        isc = rtx.InstancedScene([wl.vertices], np.zeros(2, np.uint32), maps, lo, hi)
        out = torch.empty((wl.n_rays, 4), device="cuda")
        ids = torch.empty((wl.n_rays,), dtype=torch.int32, device="cuda")

        def launch():
            isc.trace(rays, "procedural", out=out, inst_ids=ids, workspace=ws)
        outs = (out, ids)
    elif query == "multi":
        out = torch.empty((wl.n_rays, 3, 4), device="cuda")

        def launch():
            rtx.trace(sc, rays, "alpha", query="multi", k=3, out=out, workspace=ws)
        outs = (out,)
    else:
        out = torch.empty((wl.n_rays, 4) if query == "closest" else (wl.n_rays,),
                          dtype=torch.float32 if query == "closest" else torch.int32,
                          device="cuda")

        def launch():
            rtx.trace(sc, rays, "alpha", query=query, out=out, workspace=ws)
        outs = (out,)
    launch()
    torch.cuda.synchronize()
    eager = [o.clone() for o in outs]
    # the workspace has its final size before capture; warm up on the side stream
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        launch()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        launch()
    for rep in range(3):
        for o in outs:
            o.fill_(-1)
        rtx.trace(sc, rays[:100], "default")      # unrelated eager work
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert same_bits(o, e), (query, rep)


@pytest.mark.parametrize("seed", range(4))
def test_random_batches_bit_exact(env, oracle_lib, seed):
    torch, rtx = env
    rng = np.random.default_rng(9000 + seed)
    kind = ["default", "alpha", "procedural", "alpha"][seed]
    n_scenes = int(rng.integers(2, 10))
    scenes = []
    for i in range(n_scenes):
        _, v, r = random_case(100 * seed + i)
        kw = _scene_params(rng, kind, v.shape[0])
        scenes.append((v, r, kw))
    announce(f"random batch seed={seed} kind={kind} scenes={n_scenes} "
             f"rays={sum(r.shape[0] for _, r, _ in scenes)}")
    sc_list = [rtx.upload_scene(v, kw.get("geom_ids"), kw.get("texcoords"), kw.get("textures"))
               for v, _, kw in scenes]
    # per-scene alpha thresholds travel in the scene table
    batch = rtx.Batch(sc_list, [r.shape[0] for _, r, _ in scenes], kind,
                      alpha_min=[kw.get("alpha_min", 128) for _, _, kw in scenes])
    rays = torch.from_numpy(np.concatenate([r for _, r, _ in scenes])).cuda()
    checker_n = scenes[0][2].get("checker_n", 8)
    hits, cnt = batch.trace(rays, count=True, checker_n=checker_n)
    torch.cuda.synchronize()
    g = P.hits_to_numpy(hits)
    c = cnt.cpu().numpy().view(np.uint32)
    off = batch.offsets
    for i, (v, r, kw) in enumerate(scenes):
        if kind == "procedural":
            kw = dict(checker_n=checker_n)
        B = oracle_lib.traverse(v, oracle_lib.build_bvh(v), r, kind, **kw)
        sl = slice(off[i], off[i + 1])
        P.assert_exact_vs_b({k: x[sl] for k, x in g.items()}, B, f"random batch {seed} scene {i}")
        assert np.array_equal(c[sl], B["counters"]), (seed, i)
