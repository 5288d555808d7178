"""GPU parity of the 48-byte packed-reference node layout (child references
in the low bytes of moved box words, rt_bvh_pack) against oracle B's packed
traversal, bit for bit (hits, occluders, multi-hit lists, counters), and
against the float64 definition; the float32-box layout's answers on the same
rays; batched launches.  The layout is not in the paper, whose node format
is open."""
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
def tiny_f32p(env, oracle_lib):
    torch, rtx = env
    wl = W.tiny()
    ai = tiny_alpha_inputs(wl.n_tris)
    sc = rtx.upload_scene(wl.vertices, ai["geom_ids"], ai["texcoords"], ai["textures"], layout="f32p")
    assert sc.info.layout == 3
    return wl, ai, sc, oracle_lib.build_bvh(wl.vertices)


@pytest.mark.parametrize("kind", ["default", "alpha", "procedural"])
@pytest.mark.parametrize("query", ["closest", "any", "multi"])
def test_tiny_f32p_parity(env, oracle_lib, tiny_f32p, kind, query):
    torch, rtx = env
    wl, ai, sc, bvh = tiny_f32p
    announce(f"tiny f32p kind={kind} query={query}")
    okw = kind_kwargs(kind, ai)
    k = 3 if query == "multi" else 0
    B = oracle_lib.traverse(wl.vertices, bvh, wl.rays, kind, any_hit=(query == "any"), multi_k=k,
                            layout="f32p", **okw)
    rays = torch.from_numpy(wl.rays).cuda()
    out, cnt = rtx.trace(sc, rays, kind, query=query, k=max(k, 1), count=True, **trace_kwargs(kind))
    plain = rtx.trace(sc, rays, kind, query=query, k=max(k, 1), **trace_kwargs(kind))
    torch.cuda.synchronize()
    P.assert_counters_vs_b(cnt, B, f"tiny f32p {kind} {query}")
    if query == "closest":
        g = P.hits_to_numpy(out)
        P.assert_exact_vs_b(g, B, f"tiny f32p {kind}")
        assert same_bits(plain, out)
        A = oracle_lib.brute(wl.vertices, wl.rays, kind, **okw)
        P.compare_vs_a(g, A, np.arange(wl.n_rays), f"tiny f32p {kind}")
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


def test_tiny_f32p_launch_shapes(env, oracle_lib, tiny_f32p):
    """Packed-reference scenes run with the default launch shape and its
    variant without the queue (the same bits); the other compiled shapes and
    the run-time dispatch variants refuse them."""
    torch, rtx = env
    wl, ai, sc, bvh = tiny_f32p
    shapes = [tuple(s) for s in rtx.rt_launch_shapes()]
    rays = torch.from_numpy(wl.rays).cuda()
    for shape in shapes[1:]:
        if shape == (64, 8, 64, 0):
            continue
        with pytest.raises(rtx.RtxError, match="packed node layout"):
            rtx.trace(sc, rays, "alpha", alpha_min=128, shape=shape)
    from tests.test_gpu_dispatch import trace_flags
    for flags in (rtx.RT_FLAG_RUNTIME_SWITCH, rtx.RT_FLAG_RUNTIME_CALL):
        with pytest.raises(rtx.RtxError, match="compile-time intersectors"):
            trace_flags(torch, rtx, sc, rays, "alpha", flags)
    announce("tiny f32p alpha, both compiled shapes after refusals")
    okw = kind_kwargs("alpha", ai)
    B = oracle_lib.traverse(wl.vertices, bvh, wl.rays, "alpha", layout="f32p", **okw)
    for shape in ((64, 8, 64, 1), (64, 8, 64, 0)):
        for query in ("closest", "multi"):
            out, cnt = rtx.trace(sc, rays, "alpha", alpha_min=128, shape=shape, query=query, k=3,
                                 count=True)
            ref, rc = rtx.trace(sc, rays, "alpha", alpha_min=128, query=query, k=3, count=True)
            torch.cuda.synchronize()
            if query == "closest":
                P.assert_exact_vs_b(P.hits_to_numpy(out), B, f"tiny f32p {shape}")
                P.assert_counters_vs_b(cnt, B, f"tiny f32p {shape}")
            else:
                assert same_bits(out[0], ref[0]) and same_bits(out[1], ref[1])
                assert same_bits(cnt, rc)


@pytest.mark.parametrize("seed", range(6))
def test_random_scene_f32p_bit_exact(env, oracle_lib, seed):
    """The random sweep's scenes (duplicates, slivers, zero-area triangles,
    axis-aligned and tiny direction components, finite intervals) through
    the packed-reference layout."""
    torch, rtx = env
    rng, verts, rays = random_case(100 + seed)
    kind = ["default", "alpha", "procedural"][seed % 3]
    query = ["closest", "any"][(seed // 3) % 2]
    kw = _scene_params(rng, kind, verts.shape[0])
    announce(f"random f32p seed={seed} tris={verts.shape[0]} rays={rays.shape[0]} kind={kind} "
             f"query={query}")
    sc = rtx.upload_scene(verts, kw.get("geom_ids"), kw.get("texcoords"), kw.get("textures"),
                          layout="f32p")
    tkw = {kk: kw[kk] for kk in ("alpha_min", "checker_n") if kk in kw}
    out, cnt = rtx.trace(sc, torch.from_numpy(rays).cuda(), kind, query=query, count=True, **tkw)
    torch.cuda.synchronize()
    bvh = oracle_lib.build_bvh(verts)
    B = oracle_lib.traverse(verts, bvh, rays, kind, any_hit=(query == "any"), layout="f32p", **kw)
    P.assert_counters_vs_b(cnt, B, f"random f32p {seed}")
    if query == "closest":
        P.assert_exact_vs_b(P.hits_to_numpy(out), B, f"random f32p {seed}")
    else:
        assert np.array_equal(P.occluders_to_numpy(out), B["prim"])


def test_empty_and_root_leaf_f32p(env, oracle_lib):
    torch, rtx = env
    rng = np.random.default_rng(9)
    rays = np.zeros((100, 8), np.float32)
    rays[:, :3] = rng.uniform(-1, 2, size=(100, 3))
    rays[:, 4:7] = np.array([0.0, 0.0, -1.0])
    rays[:, 7] = np.inf
    for n in (0, 1, 4):
        verts = rng.uniform(0, 1, size=(n, 3, 3)).astype(np.float32)
        announce(f"f32p scene with {n} triangles")
        sc = rtx.upload_scene(verts, layout="f32p")
        hits, cnt = rtx.trace(sc, torch.from_numpy(rays).cuda(), count=True)
        torch.cuda.synchronize()
        bvh = oracle_lib.build_bvh(verts)
        B = oracle_lib.traverse(verts, bvh, rays, layout="f32p")
        P.assert_exact_vs_b(P.hits_to_numpy(hits), B, f"f32p n={n}")
        P.assert_counters_vs_b(cnt, B, f"f32p n={n}")


@pytest.fixture(scope="module")
def billboards_f32p(env, oracle_lib):
    torch, rtx = env
    wl = W.billboards()
    f32 = rtx.upload_scene(wl.vertices, wl.geom_ids, wl.texcoords, wl.textures)
    f32p = rtx.upload_scene(wl.vertices, wl.geom_ids, wl.texcoords, wl.textures, layout="f32p")
    return wl, f32, f32p, oracle_lib.build_bvh(wl.vertices)


def test_billboards_full_f32p(env, oracle_lib, billboards_f32p):
    """The benchmark's alpha launch on the packed-reference layout: all 2,073,600
    rays against oracle B (hits and counters), the any-hit query, the float64
    definition on a subsample, and the float32-box layout's hits."""
    torch, rtx = env
    wl, f32, f32p, bvh = billboards_f32p
    okw = dict(geom_ids=wl.geom_ids, texcoords=wl.texcoords, textures=wl.textures, alpha_min=128)
    rays = torch.from_numpy(wl.rays).cuda()
    announce("billboards f32p alpha closest count")
    hits, cnt = rtx.trace(f32p, rays, "alpha", count=True, alpha_min=128)
    plain = rtx.trace(f32p, rays, "alpha", alpha_min=128)
    ref = rtx.trace(f32, rays, "alpha", alpha_min=128)
    torch.cuda.synchronize()
    assert same_bits(plain, hits)
    g = P.hits_to_numpy(hits)
    B = oracle_lib.traverse(wl.vertices, bvh, wl.rays, "alpha", layout="f32p", **okw)
    P.assert_exact_vs_b(g, B, "billboards f32p alpha")
    P.assert_counters_vs_b(cnt, B, "billboards f32p alpha")
    idx = W.subsample_indices(wl.n_rays, 1920, 1080, seed=W.seed_for(W.CFG_BILLBOARDS, 9),
                              stride=16, n_random=2048)
    A = oracle_lib.brute(wl.vertices, wl.rays, "alpha", ray_index=idx, **okw)
    s = P.compare_vs_a(g, A, idx, "billboards f32p alpha")
    assert s["excluded"] <= 0.01 * len(idx)
    assert s["n_uv_over_1e-5"] <= 0.001 * s["checked"]
    # same answers as the float32-box layout except among exactly tied hits
    r = P.hits_to_numpy(ref)
    diff = np.nonzero(g["prim"] != r["prim"])[0]
    assert diff.size <= 1e-4 * wl.n_rays
    assert np.array_equal(P.bits(g["t"][diff]), P.bits(r["t"][diff]))
    same = g["prim"] == r["prim"]
    assert np.array_equal(P.bits(g["t"][same]), P.bits(r["t"][same]))
    announce("billboards f32p alpha any count")
    occ, cnt = rtx.trace(f32p, rays, "alpha", query="any", count=True, alpha_min=128)
    torch.cuda.synchronize()
    Ba = oracle_lib.traverse(wl.vertices, bvh, wl.rays, "alpha", any_hit=True, layout="f32p", **okw)
    assert np.array_equal(P.occluders_to_numpy(occ), Ba["prim"])
    P.assert_counters_vs_b(cnt, Ba, "billboards f32p alpha any")
    assert np.array_equal(Ba["prim"] == MISS, B["prim"] == MISS)


def test_spheres_full_f32p_procedural(env, oracle_lib):
    torch, rtx = env
    wl = W.spheres()
    announce("spheres 1M tris f32p procedural closest count")
    sc = rtx.upload_scene(wl.vertices, layout="f32p")
    hits, cnt = rtx.trace(sc, torch.from_numpy(wl.rays).cuda(), "procedural", count=True,
                          checker_n=8)
    torch.cuda.synchronize()
    bvh = oracle_lib.build_bvh(wl.vertices)
    B = oracle_lib.traverse(wl.vertices, bvh, wl.rays, "procedural", checker_n=8, layout="f32p")
    P.assert_exact_vs_b(P.hits_to_numpy(hits), B, "spheres f32p procedural")
    P.assert_counters_vs_b(cnt, B, "spheres f32p procedural")


def test_batch_f32p(env, oracle_lib):
    """One batched launch over packed-reference scenes equals one launch per scene
    and oracle B; a batch mixing layouts is refused at packing."""
    torch, rtx = env
    scenes = small_batch(alpha=True)
    announce(f"batch of {len(scenes)} packed-reference scenes")
    sc_list = [rtx.upload_scene(s["vertices"], s["geom_ids"], s["texcoords"], s["textures"],
                                layout="f32p") for s in scenes]
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
    for i in (0, 5):
        s = scenes[i]
        B = oracle_lib.traverse(s["vertices"], oracle_lib.build_bvh(s["vertices"]), s["rays"],
                                "alpha", geom_ids=s["geom_ids"], texcoords=s["texcoords"],
                                textures=s["textures"], alpha_min=128, layout="f32p")
        sl = slice(batch.offsets[i], batch.offsets[i + 1])
        P.assert_exact_vs_b({k: v[sl] for k, v in P.hits_to_numpy(hits).items()}, B, f"batch f32p {i}")
        P.assert_counters_vs_b(cnt[sl], B, f"batch f32p scene {i}")
    mixed = [sc_list[0], rtx.upload_scene(scenes[1]["vertices"], scenes[1]["geom_ids"],
                                          scenes[1]["texcoords"], scenes[1]["textures"])]
    with pytest.raises(rtx.RtxError, match="share one node layout"):
        rtx.Batch(mixed, [scenes[0]["rays"].shape[0], scenes[1]["rays"].shape[0]], "alpha")
