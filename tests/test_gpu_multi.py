"""GPU parity of the multi-hit query (rt_trace_multi) against oracle B
(bit-exact lists, counts and counters) and oracle A (float64 definition,
outside the exception set)."""
import numpy as np
import pytest

from paper_1912_12786_amd import workloads as W
from tests import parity as P
from tests.golden.load import load, uniform_alpha_textures

pytestmark = pytest.mark.gpu
MISS = 0xFFFFFFFF


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def multi_to_numpy(out):
    hits, n_hits = out
    h = hits.detach().cpu().numpy()
    return {"t": h[..., 0].copy(), "prim": h[..., 1].view(np.uint32).copy(), "u": h[..., 2].copy(),
            "v": h[..., 3].copy(), "n_hits": n_hits.cpu().numpy().view(np.uint32).copy()}


def assert_multi_exact(g, B, what):
    assert np.array_equal(g["n_hits"], B["n_hits"]), what
    assert np.array_equal(g["prim"], B["prim"]), what
    for k in ("t", "u", "v"):
        assert np.array_equal(P.bits(g[k]), P.bits(B[k])), (what, k)


def run(torch, rtx, scene, rays_np, kind, k, count=False, **kw):
    rays = torch.from_numpy(np.ascontiguousarray(rays_np, np.float32)).cuda()
    out = rtx.trace(scene, rays, kind, query="multi", k=k, count=count, **kw)
    torch.cuda.synchronize()
    return out


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1912_12786_amd import rtx
    rtx.load_library()
    return torch, rtx


def test_golden_layers_gpu(env):
    torch, rtx = env
    fx = load("layers.json")
    for case in fx["cases"]:
        announce(f"layers k={case['k']} alpha={case['alpha']}")
        tex = uniform_alpha_textures(case["alpha"], fx["texture_size"])
        sc = rtx.upload_scene(fx["vertices"], fx["geom_ids"], fx["texcoords"], tex)
        g = multi_to_numpy(run(torch, rtx, sc, fx["rays"], "alpha", case["k"], alpha_min=128))
        n = len(case["prims"])
        assert g["n_hits"][0] == n
        assert g["prim"][0, :n].tolist() == case["prims"]
        assert g["t"][0, :n].tolist() == case["t"]
        assert np.all(g["prim"][0, n:] == MISS)


@pytest.mark.parametrize("kind", ["default", "alpha", "procedural"])
@pytest.mark.parametrize("k", [1, 3, 8])
def test_tiny_multi_parity(env, oracle_lib, kind, k):
    torch, rtx = env
    wl = W.tiny()
    rng = np.random.default_rng(77)
    tex = W.alpha_textures(4, 64, 77)
    ai = dict(geom_ids=rng.integers(0, 4, size=wl.n_tris).astype(np.uint32),
              texcoords=rng.uniform(0, 1, size=(wl.n_tris, 3, 2)).astype(np.float32), textures=tex)
    sc = rtx.upload_scene(wl.vertices, ai["geom_ids"], ai["texcoords"], ai["textures"])
    okw = dict(ai, alpha_min=128) if kind == "alpha" else (dict(checker_n=8) if kind == "procedural" else {})
    tkw = dict(alpha_min=128) if kind == "alpha" else (dict(checker_n=8) if kind == "procedural" else {})
    rays = wl.rays[:4059]
    announce(f"tiny multi kind={kind} k={k} n_rays={rays.shape[0]}")
    out, cnt = run(torch, rtx, sc, rays, kind, k, count=True, **tkw)
    g = multi_to_numpy(out)
    bvh = oracle_lib.build_bvh(wl.vertices)
    B = oracle_lib.traverse(wl.vertices, bvh, rays, kind, multi_k=k, **okw)
    assert_multi_exact(g, B, f"tiny multi {kind} k={k}")
    P.assert_counters_vs_b(cnt, B, f"tiny multi {kind} k={k}")
    A = oracle_lib.brute_multi(wl.vertices, rays, k, kind, **okw)
    ok = A["flags"] == 0
    assert np.array_equal(g["prim"][ok], A["prim"][ok])
    assert np.array_equal(g["n_hits"][ok], A["n_hits"][ok])
    if k == 1:   # k = 1 is the closest-hit query
        c = P.hits_to_numpy(rtx.trace(sc, torch.from_numpy(rays).cuda(), kind, **tkw))
        assert np.array_equal(c["prim"], g["prim"][:, 0])
        assert np.array_equal(P.bits(c["t"]), P.bits(g["t"][:, 0]))


def test_billboards_multi_full(env, oracle_lib):
    torch, rtx = env
    wl = W.billboards()
    announce("billboards 200k tris 1920x1080 alpha multi k=4")
    sc = rtx.upload_scene(wl.vertices, wl.geom_ids, wl.texcoords, wl.textures)
    g = multi_to_numpy(run(torch, rtx, sc, wl.rays, "alpha", 4, alpha_min=128))
    okw = dict(geom_ids=wl.geom_ids, texcoords=wl.texcoords, textures=wl.textures, alpha_min=128)
    bvh = oracle_lib.build_bvh(wl.vertices)
    B = oracle_lib.traverse(wl.vertices, bvh, wl.rays, "alpha", multi_k=4, count=False, **okw)
    assert_multi_exact(g, B, "billboards multi k=4")
    idx = W.subsample_indices(wl.n_rays, 1920, 1080, seed=11, stride=32, n_random=512)
    A = oracle_lib.brute_multi(wl.vertices, wl.rays[idx], 4, "alpha", **okw)
    ok = A["flags"] == 0
    assert ok.mean() > 0.9
    assert np.array_equal(g["prim"][idx][ok], A["prim"][ok])
    hit = A["prim"][ok] != MISS
    dt = np.abs(g["t"][idx][ok][hit] - A["t"][ok][hit])
    assert np.all(dt <= 1e-5 * np.abs(A["t"][ok][hit]) + 1e-6)
