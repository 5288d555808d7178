"""GPU parity: librtx kernels (through the C ABI) against the CPU oracle.

Every test is marked ``gpu``.  Bars are documented in tests/parity.py:
bit-exact against oracle B (same BVH, same float32 operation sequence),
exact prim_id outside the exception set and t/u/v within the float32 bound
against oracle A (float64 definition).
"""
import numpy as np
import pytest

from paper_1912_12786_amd import workloads as W
from tests import parity as P
from tests.golden.load import load, uniform_alpha_textures

pytestmark = pytest.mark.gpu

MISS = 0xFFFFFFFF


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1912_12786_amd import rtx
    rtx.load_library()
    return torch


@pytest.fixture(scope="module")
def rtx_mod(torch_cuda):
    from paper_1912_12786_amd import rtx
    return rtx


def same_bits(a, b):
    """Bitwise equality (hit records carry prim_id bits, NaN as floats)."""
    import torch
    return a.shape == b.shape and torch.equal(a.view(torch.int32), b.view(torch.int32))


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


def run(rtx, torch, scene, rays_np, kind="default", query="closest", count=False, **kw):
    rays = torch.from_numpy(np.ascontiguousarray(rays_np, np.float32)).cuda()
    out = rtx.trace(scene, rays, kind, query=query, count=count, **kw)
    torch.cuda.synchronize()
    return out


def tiny_alpha_inputs(n_tris, seed=77):
    rng = np.random.default_rng(seed)
    tex = W.alpha_textures(4, 64, seed)
    return dict(geom_ids=rng.integers(0, 4, size=n_tris).astype(np.uint32),
                texcoords=rng.uniform(0, 1, size=(n_tris, 3, 2)).astype(np.float32),
                textures=tex)


def kind_kwargs(kind, alpha_inputs):
    if kind == "alpha":
        return dict(alpha_inputs, alpha_min=128)
    if kind == "procedural":
        return dict(checker_n=8)
    return {}


def trace_kwargs(kind):
    if kind == "alpha":
        return dict(alpha_min=128)
    if kind == "procedural":
        return dict(checker_n=8)
    return {}


# ----------------------------------------------------------------------------
# golden closed-form cases through the GPU path
# ----------------------------------------------------------------------------
def test_golden_cases_on_gpu(torch_cuda, rtx_mod):
    torch, rtx = torch_cuda, rtx_mod
    announce("golden fixtures, closest, default/alpha/procedural")
    fx = load("quad_centre.json")
    sc = rtx.upload_scene(fx["vertices"])
    g = P.hits_to_numpy(run(rtx, torch, sc, fx["rays"]))
    for case in fx["cases"]:
        i = case["ray"]
        if case.get("miss"):
            assert g["prim"][i] == MISS
            continue
        acc = {a["prim"]: a for a in case["accept"]}
        assert int(g["prim"][i]) in acc
        a = acc[int(g["prim"][i])]
        assert (g["t"][i], g["u"][i], g["v"][i]) == (a["t"], a["u"], a["v"])
        if "oracle_b_prim" in case:
            assert g["prim"][i] == case["oracle_b_prim"]

    fx = load("shared_edge.json")
    sc = rtx.upload_scene(fx["vertices"])
    g = P.hits_to_numpy(run(rtx, torch, sc, fx["rays"]))
    assert g["prim"][0] in (0, 1) and g["t"][0] == 1.0
    assert g["prim"][1] == MISS

    fx = load("transparent_billboard.json")
    tex = uniform_alpha_textures(fx["texture_alpha"], fx["texture_size"])
    for case in fx["cases"]:
        sel = case.get("only_prims", list(range(len(fx["vertices"]))))
        sc = rtx.upload_scene(fx["vertices"][sel], fx["geom_ids"][sel], fx["texcoords"][sel], tex)
        kw = dict(alpha_min=case["alpha_min"]) if case["intersector"] == "alpha" else {}
        hits, cnt = run(rtx, torch, sc, fx["rays"], case["intersector"], count=True, **kw)
        g = P.hits_to_numpy(hits)
        if case.get("miss"):
            assert g["prim"][0] == MISS
        else:
            a = case["accept"][0]
            assert (int(g["prim"][0]), g["t"][0], g["u"][0], g["v"][0]) == (a["prim"], a["t"], a["u"], a["v"])
        assert cnt.cpu().numpy()[0].tolist() == case["counters"]

    fx = load("alpha_threshold.json")
    for case in fx["cases"]:
        tex = uniform_alpha_textures([case["a8"]], fx["texture_size"])
        sc = rtx.upload_scene(fx["vertices"], fx["geom_ids"], fx["texcoords"], tex)
        g = P.hits_to_numpy(run(rtx, torch, sc, fx["rays"], "alpha", alpha_min=case["alpha_min"]))
        assert (g["prim"][0] != MISS) == case["hit"], case

    fx = load("procedural_checker.json")
    rays = np.array([[x, y, 1, 0, 0, 0, -1, np.inf] for x, y, _ in fx["points"]], np.float32)
    sc = rtx.upload_scene(fx["vertices"])
    g = P.hits_to_numpy(run(rtx, torch, sc, rays, "procedural", checker_n=fx["checker_n"]))
    for i, (x, y, vis) in enumerate(fx["points"]):
        assert (g["prim"][i] != MISS) == vis

    fx = load("two_leaf_counts.json")
    sc = rtx.upload_scene(fx["vertices"])
    hits, cnt = run(rtx, torch, sc, fx["rays"], count=True)
    g = P.hits_to_numpy(hits)
    c = cnt.cpu().numpy()
    for case in fx["cases"]:
        i = case["ray"]
        assert c[i].tolist() == case["counters"], case
        assert (g["prim"][i] == MISS) if case.get("miss") else (g["prim"][i] == case["prim"])


# ----------------------------------------------------------------------------
# tiny workload: every intersector x query x counting, several ray counts
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def tiny_setup(torch_cuda, rtx_mod, oracle_lib):
    wl = W.tiny()
    ai = tiny_alpha_inputs(wl.n_tris)
    scene = rtx_mod.upload_scene(wl.vertices, ai["geom_ids"], ai["texcoords"], ai["textures"])
    bvh = oracle_lib.build_bvh(wl.vertices)
    return wl, ai, scene, bvh


@pytest.mark.parametrize("kind", ["default", "alpha", "procedural"])
@pytest.mark.parametrize("query", ["closest", "any"])
@pytest.mark.parametrize("n_rays", [4096, 4059, 1, 65])
def test_tiny_parity(torch_cuda, rtx_mod, oracle_lib, tiny_setup, kind, query, n_rays):
    torch, rtx = torch_cuda, rtx_mod
    wl, ai, scene, bvh = tiny_setup
    rays = wl.rays[:n_rays] if n_rays != 65 else wl.rays[1000:1065]
    announce(f"tiny kind={kind} query={query} n_rays={rays.shape[0]} count=True")
    okw = kind_kwargs(kind, ai)
    B = oracle_lib.traverse(wl.vertices, bvh, rays, kind, any_hit=(query == "any"), **okw)
    out, cnt = run(rtx, torch, scene, rays, kind, query=query, count=True, **trace_kwargs(kind))
    P.assert_counters_vs_b(cnt, B, f"tiny {kind} {query}")
    # the non-counting instantiation must agree with the counting one
    plain = run(rtx, torch, scene, rays, kind, query=query, count=False, **trace_kwargs(kind))
    if query == "closest":
        g = P.hits_to_numpy(out)
        P.assert_exact_vs_b(g, B, f"tiny {kind}")
        assert same_bits(plain, out)
        A = oracle_lib.brute(wl.vertices, rays, kind, **okw)
        P.compare_vs_a(g, A, np.arange(rays.shape[0]), f"tiny {kind}")
    else:
        occ = P.occluders_to_numpy(out)
        assert np.array_equal(occ, B["prim"])
        assert same_bits(plain, out)
        A = oracle_lib.brute(wl.vertices, rays, kind, any_hit=True, **okw)
        P.compare_vs_a({"prim": occ}, A, np.arange(rays.shape[0]), f"tiny {kind} any", any_hit=True)


def test_tiny_all_launch_shapes_identical(torch_cuda, rtx_mod, tiny_setup):
    torch, rtx = torch_cuda, rtx_mod
    wl, ai, scene, _ = tiny_setup
    shapes = rtx.rt_launch_shapes()
    ref = None
    for shape in shapes:
        announce(f"tiny alpha count shape={shape}")
        hits, cnt = run(rtx, torch, scene, wl.rays, "alpha", count=True, alpha_min=128, shape=shape)
        if ref is None:
            ref = (hits, cnt)
        else:
            assert same_bits(hits, ref[0]) and same_bits(cnt, ref[1])


# ----------------------------------------------------------------------------
# edge cases
# ----------------------------------------------------------------------------
def test_empty_scene_gpu(torch_cuda, rtx_mod):
    torch, rtx = torch_cuda, rtx_mod
    announce("empty scene")
    sc = rtx.upload_scene(np.zeros((0, 3, 3), np.float32))
    rays = W.tiny().rays[:100]
    hits, cnt = run(rtx, torch, sc, rays, count=True)
    g = P.hits_to_numpy(hits)
    assert np.all(g["prim"] == MISS) and np.all(np.isinf(g["t"]))
    assert np.all(g["u"] == 0) and np.all(g["v"] == 0)
    assert np.all(cnt.cpu().numpy() == 0)
    occ = run(rtx, torch, sc, rays, query="any")
    assert np.all(P.occluders_to_numpy(occ) == MISS)


def test_degenerate_rays_and_small_scenes(torch_cuda, rtx_mod, oracle_lib):
    torch, rtx = torch_cuda, rtx_mod
    rng = np.random.default_rng(21)
    for n_tris in (1, 2, 4, 5, 33):
        announce(f"degenerate rays, n_tris={n_tris}")
        verts = rng.uniform(-1, 1, size=(n_tris, 3, 3)).astype(np.float32)
        rays = []
        for _ in range(200):
            o = rng.uniform(-2, 2, size=3)
            d = rng.normal(size=3)
            # axis-aligned and zero components, tiny components, tmin == tmax
            m = rng.integers(0, 5)
            if m == 1:
                d[rng.integers(0, 3)] = 0.0
            elif m == 2:
                d[:] = 0.0
                d[rng.integers(0, 3)] = rng.choice([-1.0, 1.0])
            elif m == 3:
                d[rng.integers(0, 3)] = 1e-30
            tmin, tmax = 0.0, np.inf
            if rng.integers(0, 6) == 0:
                tmin = tmax = float(rng.uniform(0, 3))
            elif rng.integers(0, 6) == 0:
                tmax = float(rng.uniform(0, 3))
            rays.append([*o, tmin, *d, tmax])
        rays = np.asarray(rays, np.float32)
        bvh = oracle_lib.build_bvh(verts)
        B = oracle_lib.traverse(verts, bvh, rays)
        sc = rtx.upload_scene(verts)
        hits, cnt = run(rtx, torch, sc, rays, count=True)
        P.assert_exact_vs_b(P.hits_to_numpy(hits), B, f"degenerate n={n_tris}")
        P.assert_counters_vs_b(cnt, B, f"degenerate n={n_tris}")


def deep_scene(n=160):
    """Triangles in the planes x = k, all around the x axis, growing by 1.5x
    per step: the surface-area cost always prefers to split off the few
    largest ones, so the BVH reaches the depth-40 median fallback -- far deeper
    than the on-chip stack."""
    s = (1.5 ** np.arange(n)).astype(np.float64)
    v = np.zeros((n, 3, 3), np.float64)
    v[:, :, 0] = np.arange(n)[:, None]
    v[:, 0, 1], v[:, 0, 2] = -s, -s
    v[:, 1, 1], v[:, 1, 2] = 2 * s, -s
    v[:, 2, 1], v[:, 2, 2] = -s, 2 * s
    return v.astype(np.float32)


def test_deep_bvh_uses_spill_stack(torch_cuda, rtx_mod, oracle_lib):
    torch, rtx = torch_cuda, rtx_mod
    verts = deep_scene()
    bvh = oracle_lib.build_bvh(verts)
    assert bvh.max_depth > 30
    n = verts.shape[0]
    tex = uniform_alpha_textures([0], (2, 2))
    ai = dict(geom_ids=np.zeros(n, np.uint32), texcoords=np.zeros((n, 3, 2), np.float32),
              textures=tex)
    sc = rtx.upload_scene(verts, ai["geom_ids"], ai["texcoords"], tex)
    rng = np.random.default_rng(3)
    rays = np.zeros((300, 8), np.float32)
    rays[:, 0] = -1.0
    rays[:, 1:3] = rng.uniform(-0.2, 0.2, size=(300, 2))
    rays[:, 4] = 1.0
    rays[150:, 5:7] = rng.normal(0, 1e-3, size=(150, 2))
    rays[:, 7] = np.inf
    shapes = rtx.rt_launch_shapes()
    for i, shape in enumerate(shapes):
        assert rtx.rt_trace_workspace_bytes(sc.view, 300, rtx.RT_FLAG_SHAPE(i)) > 0
        for kind, kw in (("alpha", dict(alpha_min=1)), ("default", {})):
            announce(f"deep bvh kind={kind} shape={shape}")
            okw = dict(ai, alpha_min=1) if kind == "alpha" else {}
            B = oracle_lib.traverse(verts, bvh, rays, kind, **okw)
            hits, cnt = run(rtx, torch, sc, rays, kind, count=True, shape=shape, **kw)
            P.assert_exact_vs_b(P.hits_to_numpy(hits), B, f"deep {kind}")
            P.assert_counters_vs_b(cnt, B, f"deep {kind}")
            if kind == "alpha":   # every box along the ray visited
                assert B["counters"][:, 1].max() == n


def test_nondefault_stream_and_determinism(torch_cuda, rtx_mod, tiny_setup):
    torch, rtx = torch_cuda, rtx_mod
    wl, ai, scene, _ = tiny_setup
    announce("tiny alpha on a side stream, repeated")
    rays = torch.from_numpy(wl.rays).cuda()
    ref = rtx.trace(scene, rays, "alpha", alpha_min=128)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        outs = [rtx.trace(scene, rays, "alpha", alpha_min=128) for _ in range(5)]
    s.synchronize()
    for o in outs:
        assert same_bits(o, ref)


# ----------------------------------------------------------------------------
# full-size workloads (the benchmark's launch configuration)
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def billboards_setup(torch_cuda, rtx_mod, oracle_lib):
    wl = W.billboards()
    scene = rtx_mod.upload_scene(wl.vertices, wl.geom_ids, wl.texcoords, wl.textures)
    bvh = oracle_lib.build_bvh(wl.vertices)
    idx = W.subsample_indices(wl.n_rays, 1920, 1080, seed=W.seed_for(W.CFG_BILLBOARDS, 9),
                              stride=8, n_random=8192)
    return wl, scene, bvh, idx


@pytest.mark.parametrize("kind", ["alpha", "default"])
def test_billboards_full_closest(torch_cuda, rtx_mod, oracle_lib, billboards_setup, kind):
    torch, rtx = torch_cuda, rtx_mod
    wl, scene, bvh, idx = billboards_setup
    okw = dict(geom_ids=wl.geom_ids, texcoords=wl.texcoords, textures=wl.textures,
               alpha_min=128) if kind == "alpha" else {}
    announce(f"billboards 200k tris 1920x1080 kind={kind} closest (bench launch shape)")
    hits = run(rtx, torch, scene, wl.rays, kind, **trace_kwargs(kind))
    g = P.hits_to_numpy(hits)
    B = oracle_lib.traverse(wl.vertices, bvh, wl.rays, kind, count=False, **okw)
    P.assert_exact_vs_b(g, B, f"billboards {kind}")
    A = oracle_lib.brute(wl.vertices, wl.rays, kind, ray_index=idx, **okw)
    s = P.compare_vs_a(g, A, idx, f"billboards {kind}")
    print("oracle A summary", kind, s, flush=True)
    # measured on these rays: 267 (alpha) and 25 (default) of 40,450 in the
    # exception set; 12 and 7 rays with a u/v error above 1e-5 that pass only
    # through the widened float32 bound
    assert s["excluded"] <= 0.01 * len(idx)
    assert s["n_uv_over_1e-5"] <= 0.001 * s["checked"]


def test_billboards_full_counts_and_any(torch_cuda, rtx_mod, oracle_lib, billboards_setup):
    torch, rtx = torch_cuda, rtx_mod
    wl, scene, bvh, idx = billboards_setup
    okw = dict(geom_ids=wl.geom_ids, texcoords=wl.texcoords, textures=wl.textures, alpha_min=128)
    announce("billboards alpha closest count")
    hits, cnt = run(rtx, torch, scene, wl.rays, "alpha", count=True, alpha_min=128)
    B = oracle_lib.traverse(wl.vertices, bvh, wl.rays, "alpha", **okw)
    P.assert_exact_vs_b(P.hits_to_numpy(hits), B, "billboards alpha count")
    P.assert_counters_vs_b(cnt, B, "billboards alpha count")
    announce("billboards alpha any count")
    occ, cnt = run(rtx, torch, scene, wl.rays, "alpha", query="any", count=True, alpha_min=128)
    Ba = oracle_lib.traverse(wl.vertices, bvh, wl.rays, "alpha", any_hit=True, **okw)
    assert np.array_equal(P.occluders_to_numpy(occ), Ba["prim"])
    P.assert_counters_vs_b(cnt, Ba, "billboards alpha any count")
    # occluded <=> closest hit exists
    assert np.array_equal(Ba["prim"] == MISS, B["prim"] == MISS)


@pytest.fixture(scope="module")
def spheres_setup(torch_cuda, rtx_mod, oracle_lib):
    wl = W.spheres()
    scene = rtx_mod.upload_scene(wl.vertices)
    bvh = oracle_lib.build_bvh(wl.vertices)
    return wl, scene, bvh


def test_spheres_full_procedural_counts(torch_cuda, rtx_mod, oracle_lib, spheres_setup):
    torch, rtx = torch_cuda, rtx_mod
    wl, scene, bvh = spheres_setup
    announce("spheres 1M tris, primary+bounce, procedural closest count")
    hits, cnt = run(rtx, torch, scene, wl.rays, "procedural", count=True, checker_n=8)
    B = oracle_lib.traverse(wl.vertices, bvh, wl.rays, "procedural", checker_n=8)
    g = P.hits_to_numpy(hits)
    P.assert_exact_vs_b(g, B, "spheres procedural")
    P.assert_counters_vs_b(cnt, B, "spheres procedural")
    idx = W.subsample_indices(wl.n_rays, None, None, seed=W.seed_for(W.CFG_SPHERES, 9),
                              n_random=8192)
    A = oracle_lib.brute(wl.vertices, wl.rays, "procedural", ray_index=idx, checker_n=8)
    s = P.compare_vs_a(g, A, idx, "spheres procedural")
    print("oracle A summary spheres", s, flush=True)
    # measured: 133 of 8,183 in the exception set (131 near a checker line:
    # small far triangles widen the float32 bound and so the band), and 240
    # rays with a u/v error above 1e-5 within their bound (triangles about
    # 1/1000 of their distance wide)
    assert s["excluded"] <= 0.025 * len(idx)
    assert s["n_uv_over_1e-5"] <= 0.05 * s["checked"]
    announce("spheres default closest count")
    hits, cnt = run(rtx, torch, scene, wl.rays, "default", count=True)
    B = oracle_lib.traverse(wl.vertices, bvh, wl.rays, "default")
    P.assert_exact_vs_b(P.hits_to_numpy(hits), B, "spheres default")
    P.assert_counters_vs_b(cnt, B, "spheres default")
