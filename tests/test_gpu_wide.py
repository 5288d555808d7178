"""GPU parity of the four-wide node layout (rt_bvh_widen: 128-B nodes of up
to four children collapsed from the binary BVH) against oracle B's wide
traversal, bit for bit (hits, occluders, multi-hit lists, counters), in both
compiled launch shapes (8 and 16 LDS stack slots), against the float64
definition, against the binary layout's answers on the same rays, and in
batched launches.  The layout is not in the paper, which leaves the BVH's
arity open."""
import numpy as np
import pytest

from paper_1912_12786_amd import workloads as W
from tests import parity as P
from tests.test_gpu_batch import small_batch
from tests.test_gpu_parity import kind_kwargs, tiny_alpha_inputs, trace_kwargs
from tests.test_gpu_random import random_case
from tests.test_oracle_pins import _scene_params

pytestmark = pytest.mark.gpu
MISS = 0xFFFFFFFF
WIDE_SHAPES = [(64, 8, 64, 1), (64, 16, 64, 1)]


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


@pytest.fixture(scope="module")
def tiny_wide(env, oracle_lib):
    torch, rtx = env
    wl = W.tiny()
    ai = tiny_alpha_inputs(wl.n_tris)
    sc = rtx.upload_scene(wl.vertices, ai["geom_ids"], ai["texcoords"], ai["textures"],
                          layout="wide4")
    assert sc.info.layout == 2
    return wl, ai, sc, oracle_lib.build_bvh(wl.vertices)


@pytest.mark.parametrize("shape", WIDE_SHAPES)
@pytest.mark.parametrize("kind", ["default", "alpha", "procedural"])
@pytest.mark.parametrize("query", ["closest", "any", "multi"])
def test_tiny_wide_parity(env, oracle_lib, tiny_wide, kind, query, shape):
    torch, rtx = env
    wl, ai, sc, bvh = tiny_wide
    announce(f"tiny wide4 kind={kind} query={query} shape={shape}")
    okw = kind_kwargs(kind, ai)
    k = 3 if query == "multi" else 0
    B = oracle_lib.traverse(wl.vertices, bvh, wl.rays, kind, any_hit=(query == "any"), multi_k=k,
                            layout="wide4", **okw)
    rays = torch.from_numpy(wl.rays).cuda()
    out, cnt = rtx.trace(sc, rays, kind, query=query, k=max(k, 1), count=True, shape=shape,
                         **trace_kwargs(kind))
    plain = rtx.trace(sc, rays, kind, query=query, k=max(k, 1), shape=shape, **trace_kwargs(kind))
    torch.cuda.synchronize()
    P.assert_counters_vs_b(cnt, B, f"tiny wide4 {kind} {query}")
    if query == "closest":
        g = P.hits_to_numpy(out)
        P.assert_exact_vs_b(g, B, f"tiny wide4 {kind}")
        assert same_bits(plain, out)
        A = oracle_lib.brute(wl.vertices, wl.rays, kind, **okw)
        P.compare_vs_a(g, A, np.arange(wl.n_rays), f"tiny wide4 {kind}")
    elif query == "any":
        assert np.array_equal(P.occluders_to_numpy(out), B["prim"])
        assert same_bits(plain, out)
    else:
        hits, nh = out
        h = hits.cpu().numpy()
        assert np.array_equal(nh.cpu().numpy().view(np.uint32), B["n_hits"])
        assert np.array_equal(np.ascontiguousarray(h[..., 1]).view(np.uint32),
                              np.asarray(B["prim"], np.uint32).reshape(-1, k))
        for col, key in ((0, "t"), (2, "u"), (3, "v")):
            assert np.array_equal(h[..., col].view(np.uint32),
                                  np.ascontiguousarray(B[key], np.float32).reshape(-1, k).view(np.uint32))
        assert same_bits(plain[0], hits)


def test_tiny_wide_refused_shapes(env, tiny_wide):
    """Four-wide scenes run with the two compiled shapes; the other shapes
    and the run-time dispatch variants refuse them before launching."""
    torch, rtx = env
    wl, ai, sc, _ = tiny_wide
    rays = torch.from_numpy(wl.rays).cuda()
    for shape in rtx.rt_launch_shapes():
        if tuple(shape) in WIDE_SHAPES:
            continue
        with pytest.raises(rtx.RtxError, match="four-wide"):
            rtx.trace(sc, rays, "alpha", alpha_min=128, shape=shape)
    from tests.test_gpu_dispatch import trace_flags
    for flags in (rtx.RT_FLAG_RUNTIME_SWITCH, rtx.RT_FLAG_RUNTIME_CALL):
        with pytest.raises(rtx.RtxError, match="compile-time intersectors"):
            trace_flags(torch, rtx, sc, rays, "alpha", flags)


@pytest.mark.parametrize("seed", range(6))
def test_random_scene_wide_bit_exact(env, oracle_lib, seed):
    """The random sweep's scenes (duplicates, slivers, zero-area triangles,
    axis-aligned and tiny direction components, finite intervals) through
    the four-wide layout, leaves of 1 to 4 triangles."""
    torch, rtx = env
    rng, verts, rays = random_case(300 + seed)
    kind = ["default", "alpha", "procedural"][seed % 3]
    query = ["closest", "any"][(seed // 3) % 2]
    max_leaf = 1 + seed % 4
    kw = _scene_params(rng, kind, verts.shape[0])
    shape = WIDE_SHAPES[seed % 2]
    announce(f"random wide4 seed={seed} tris={verts.shape[0]} rays={rays.shape[0]} kind={kind} "
             f"query={query} leaf={max_leaf} shape={shape}")
    sc = rtx.upload_scene(verts, kw.get("geom_ids"), kw.get("texcoords"), kw.get("textures"),
                          layout="wide4", max_leaf=max_leaf)
    tkw = {kk: kw[kk] for kk in ("alpha_min", "checker_n") if kk in kw}
    out, cnt = rtx.trace(sc, torch.from_numpy(rays).cuda(), kind, query=query, count=True,
                         shape=shape, **tkw)
    torch.cuda.synchronize()
    bvh = oracle_lib.build_bvh(verts, max_leaf=max_leaf)
    B = oracle_lib.traverse(verts, bvh, rays, kind, any_hit=(query == "any"), layout="wide4", **kw)
    P.assert_counters_vs_b(cnt, B, f"random wide4 {seed}")
    if query == "closest":
        P.assert_exact_vs_b(P.hits_to_numpy(out), B, f"random wide4 {seed}")
    else:
        assert np.array_equal(P.occluders_to_numpy(out), B["prim"])


def test_empty_root_leaf_and_deep_wide(env, oracle_lib):
    """Empty scenes and root leaves (no wide node), and a deep stack that
    spills past both LDS rings: 4,096 triangles stacked along z with leaves
    of one triangle, rays straight down through all of them."""
    torch, rtx = env
    rng = np.random.default_rng(9)
    rays = np.zeros((100, 8), np.float32)
    rays[:, :3] = rng.uniform(-1, 2, size=(100, 3))
    rays[:, 4:7] = np.array([0.0, 0.0, -1.0])
    rays[:, 7] = np.inf
    for n in (0, 1, 4):
        verts = rng.uniform(0, 1, size=(n, 3, 3)).astype(np.float32)
        announce(f"wide4 scene with {n} triangles")
        sc = rtx.upload_scene(verts, layout="wide4")
        assert sc.info.n_nodes == 0
        hits, cnt = rtx.trace(sc, torch.from_numpy(rays).cuda(), count=True)
        torch.cuda.synchronize()
        B = oracle_lib.traverse(verts, oracle_lib.build_bvh(verts), rays, layout="wide4")
        P.assert_exact_vs_b(P.hits_to_numpy(hits), B, f"wide4 n={n}")
        P.assert_counters_vs_b(cnt, B, f"wide4 n={n}")
    n = 4096
    z = np.sort(rng.uniform(0, 10, n)).astype(np.float32)
    v = np.zeros((n, 3, 3), np.float32)
    v[:, 0, 2] = v[:, 1, 2] = v[:, 2, 2] = z
    v[:, 1, 0] = 1.0
    v[:, 2, 1] = 1.0
    sc = rtx.upload_scene(v, layout="wide4", max_leaf=1)
    assert sc.info.max_depth > 15, sc.info.max_depth
    m = 5000
    r = np.zeros((m, 8), np.float32)
    r[:, 0:2] = rng.uniform(0.01, 0.49, size=(m, 2))
    r[:, 2] = 11.0
    r[:, 6] = -1.0
    r[:, 7] = np.inf
    r[::2, 3] = rng.uniform(0, 11, size=(m + 1) // 2)   # half the rays start below some slabs
    bvh = oracle_lib.build_bvh(v, max_leaf=1)
    for query in ("closest", "any"):
        B = oracle_lib.traverse(v, bvh, r, any_hit=(query == "any"), layout="wide4")
        for shape in WIDE_SHAPES:
            announce(f"deep wide4 stack {sc.info.max_depth} query={query} shape={shape}")
            out, cnt = rtx.trace(sc, torch.from_numpy(r).cuda(), query=query, count=True,
                                 shape=shape)
            torch.cuda.synchronize()
            P.assert_counters_vs_b(cnt, B, f"deep wide4 {query} {shape}")
            if query == "closest":
                P.assert_exact_vs_b(P.hits_to_numpy(out), B, f"deep wide4 {shape}")
            else:
                assert np.array_equal(P.occluders_to_numpy(out), B["prim"])


@pytest.fixture(scope="module")
def billboards_wide(env, oracle_lib):
    torch, rtx = env
    wl = W.billboards()
    f32 = rtx.upload_scene(wl.vertices, wl.geom_ids, wl.texcoords, wl.textures, max_leaf=2)
    wide = rtx.upload_scene(wl.vertices, wl.geom_ids, wl.texcoords, wl.textures, layout="wide4",
                            max_leaf=2)
    return wl, f32, wide, oracle_lib.build_bvh(wl.vertices, max_leaf=2)


@pytest.mark.parametrize("shape", WIDE_SHAPES)
def test_billboards_full_wide(env, oracle_lib, billboards_wide, shape):
    """The benchmark's alpha launch on the four-wide layout: all 2,073,600
    rays against oracle B (hits and counters), the any-hit query, the
    float64 definition on a subsample, and the binary layout's hits."""
    torch, rtx = env
    wl, f32, wide, bvh = billboards_wide
    okw = dict(geom_ids=wl.geom_ids, texcoords=wl.texcoords, textures=wl.textures, alpha_min=128)
    rays = torch.from_numpy(wl.rays).cuda()
    announce(f"billboards wide4 alpha closest count shape={shape}")
    hits, cnt = rtx.trace(wide, rays, "alpha", count=True, alpha_min=128, shape=shape)
    plain = rtx.trace(wide, rays, "alpha", alpha_min=128, shape=shape)
    ref = rtx.trace(f32, rays, "alpha", alpha_min=128)
    torch.cuda.synchronize()
    assert same_bits(plain, hits)
    g = P.hits_to_numpy(hits)
    B = oracle_lib.traverse(wl.vertices, bvh, wl.rays, "alpha", layout="wide4", **okw)
    P.assert_exact_vs_b(g, B, "billboards wide4 alpha")
    P.assert_counters_vs_b(cnt, B, "billboards wide4 alpha")
    if shape == WIDE_SHAPES[0]:
        idx = W.subsample_indices(wl.n_rays, 1920, 1080, seed=W.seed_for(W.CFG_BILLBOARDS, 10),
                                  stride=16, n_random=2048)
        A = oracle_lib.brute(wl.vertices, wl.rays, "alpha", ray_index=idx, **okw)
        s = P.compare_vs_a(g, A, idx, "billboards wide4 alpha")
        assert s["excluded"] <= 0.01 * len(idx)
        assert s["n_uv_over_1e-5"] <= 0.001 * s["checked"]
    r = P.hits_to_numpy(ref)
    diff = np.nonzero(g["prim"] != r["prim"])[0]
    assert diff.size <= 1e-4 * wl.n_rays
    assert np.array_equal(P.bits(g["t"]), P.bits(r["t"]))
    announce(f"billboards wide4 alpha any count shape={shape}")
    occ, cnt = rtx.trace(wide, rays, "alpha", query="any", count=True, alpha_min=128, shape=shape)
    torch.cuda.synchronize()
    Ba = oracle_lib.traverse(wl.vertices, bvh, wl.rays, "alpha", any_hit=True, layout="wide4",
                             **okw)
    assert np.array_equal(P.occluders_to_numpy(occ), Ba["prim"])
    P.assert_counters_vs_b(cnt, Ba, "billboards wide4 alpha any")
    assert np.array_equal(Ba["prim"] == MISS, B["prim"] == MISS)


def test_spheres_full_wide_procedural(env, oracle_lib):
    torch, rtx = env
    wl = W.spheres()
    announce("spheres 1M tris wide4 procedural closest count")
    sc = rtx.upload_scene(wl.vertices, layout="wide4", max_leaf=2)
    hits, cnt = rtx.trace(sc, torch.from_numpy(wl.rays).cuda(), "procedural", count=True,
                          checker_n=8)
    torch.cuda.synchronize()
    bvh = oracle_lib.build_bvh(wl.vertices, max_leaf=2)
    B = oracle_lib.traverse(wl.vertices, bvh, wl.rays, "procedural", checker_n=8, layout="wide4")
    P.assert_exact_vs_b(P.hits_to_numpy(hits), B, "spheres wide4 procedural")
    P.assert_counters_vs_b(cnt, B, "spheres wide4 procedural")


def test_batch_wide(env, oracle_lib):
    """One batched launch over four-wide scenes equals one launch per scene
    and oracle B."""
    torch, rtx = env
    scenes = small_batch(alpha=True)
    announce(f"batch of {len(scenes)} four-wide scenes")
    sc_list = [rtx.upload_scene(s["vertices"], s["geom_ids"], s["texcoords"], s["textures"],
                                layout="wide4") for s in scenes]
    batch = rtx.Batch(sc_list, [s["rays"].shape[0] for s in scenes], "alpha")
    rays = torch.from_numpy(np.concatenate([s["rays"] for s in scenes])).cuda()
    hits, cnt = batch.trace(rays, count=True)
    outs, cnts = [], []
    for sc, s in zip(sc_list, scenes):
        h, c = rtx.trace(sc, torch.from_numpy(s["rays"]).cuda(), "alpha", count=True, alpha_min=128)
        outs.append(h)
        cnts.append(c)
    torch.cuda.synchronize()
    assert same_bits(hits, torch.cat(outs)) and same_bits(cnt, torch.cat(cnts))
    g = P.hits_to_numpy(hits)
    c_all = cnt.cpu()
    for i, s in enumerate(scenes):
        B = oracle_lib.traverse(s["vertices"], oracle_lib.build_bvh(s["vertices"]), s["rays"],
                                "alpha", geom_ids=s["geom_ids"], texcoords=s["texcoords"],
                                textures=s["textures"], alpha_min=128, layout="wide4")
        sl = slice(batch.offsets[i], batch.offsets[i + 1])
        P.assert_exact_vs_b({k: v[sl] for k, v in g.items()}, B, f"batch wide4 {i}")
        P.assert_counters_vs_b(c_all[sl], B, f"batch wide4 scene {i}")
