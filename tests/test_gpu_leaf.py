"""GPU parity for BVHs built with other leaf size limits (rt_bvh_build_ex):
every compiled kernel against oracle B built with the same limit, bit for
bit (hits, occluders, counters), including the benchmark's configuration
(billboards, leaves of at most 2 triangles, both node layouts)."""
import numpy as np
import pytest

from paper_1912_12786_amd import workloads as W
from tests import parity as P
from tests.test_gpu_parity import kind_kwargs, tiny_alpha_inputs, trace_kwargs

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


@pytest.mark.parametrize("max_leaf", [1, 2, 7])
@pytest.mark.parametrize("kind", ["alpha", "procedural"])
@pytest.mark.parametrize("query", ["closest", "any"])
def test_tiny_leaf_sizes(env, oracle_lib, max_leaf, kind, query):
    torch, rtx = env
    wl = W.tiny()
    ai = tiny_alpha_inputs(wl.n_tris)
    announce(f"tiny max_leaf={max_leaf} kind={kind} query={query}")
    sc = rtx.upload_scene(wl.vertices, ai["geom_ids"], ai["texcoords"], ai["textures"],
                          max_leaf=max_leaf)
    assert sc.info.max_leaf == max_leaf
    out, cnt = rtx.trace(sc, torch.from_numpy(wl.rays).cuda(), kind, query=query, count=True,
                         **trace_kwargs(kind))
    torch.cuda.synchronize()
    bvh = oracle_lib.build_bvh(wl.vertices, max_leaf=max_leaf)
    B = oracle_lib.traverse(wl.vertices, bvh, wl.rays, kind, any_hit=(query == "any"),
                            **kind_kwargs(kind, ai))
    P.assert_counters_vs_b(cnt, B, f"tiny leaf {max_leaf}")
    if query == "closest":
        P.assert_exact_vs_b(P.hits_to_numpy(out), B, f"tiny leaf {max_leaf} {kind}")
    else:
        assert np.array_equal(P.occluders_to_numpy(out), B["prim"])


@pytest.mark.parametrize("layout", ["f32", "q8"])
def test_billboards_bench_config(env, oracle_lib, layout):
    """The benchmark's launch (alpha, billboards, 1920x1080, leaves of at
    most 2 triangles): all rays against oracle B with hits and counters, the
    float64 definition on a subsample."""
    torch, rtx = env
    wl = W.billboards()
    announce(f"billboards alpha max_leaf=2 layout={layout}")
    sc = rtx.upload_scene(wl.vertices, wl.geom_ids, wl.texcoords, wl.textures, max_leaf=2,
                          layout=layout)
    rays = torch.from_numpy(wl.rays).cuda()
    hits, cnt = rtx.trace(sc, rays, "alpha", count=True, alpha_min=128)
    plain = rtx.trace(sc, rays, "alpha", alpha_min=128)
    torch.cuda.synchronize()
    assert torch.equal(plain.view(torch.int32), hits.view(torch.int32))
    okw = dict(geom_ids=wl.geom_ids, texcoords=wl.texcoords, textures=wl.textures, alpha_min=128)
    bvh = oracle_lib.build_bvh(wl.vertices, max_leaf=2)
    B = oracle_lib.traverse(wl.vertices, bvh, wl.rays, "alpha", layout=layout, **okw)
    g = P.hits_to_numpy(hits)
    P.assert_exact_vs_b(g, B, f"billboards leaf 2 {layout}")
    P.assert_counters_vs_b(cnt, B, f"billboards leaf 2 {layout}")
    idx = W.subsample_indices(wl.n_rays, 1920, 1080, seed=W.seed_for(W.CFG_BILLBOARDS, 9),
                              stride=16, n_random=2048)
    A = oracle_lib.brute(wl.vertices, wl.rays, "alpha", ray_index=idx, **okw)
    s = P.compare_vs_a(g, A, idx, f"billboards leaf 2 {layout}")
    assert s["excluded"] <= 0.01 * len(idx)
    assert s["n_uv_over_1e-5"] <= 0.001 * s["checked"]
    announce(f"billboards alpha any max_leaf=2 layout={layout}")
    occ = rtx.trace(sc, rays, "alpha", query="any", alpha_min=128)
    torch.cuda.synchronize()
    Ba = oracle_lib.traverse(wl.vertices, bvh, wl.rays, "alpha", any_hit=True, layout=layout,
                             count=False, **okw)
    assert np.array_equal(P.occluders_to_numpy(occ), Ba["prim"])


def test_tune_scene_chooses_a_build_and_shape(env, oracle_lib, tmp_path):
    """The autotuner over leaf size x node layout x launch shape returns a
    scene built the chosen way; its results equal oracle B built the same
    way; a second call reuses the cached choice."""
    torch, rtx = env
    from paper_1912_12786_amd import autotune
    wl = W.tiny()
    ai = tiny_alpha_inputs(wl.n_tris)
    rays = torch.from_numpy(wl.rays).cuda()
    cache = str(tmp_path / "tune.json")
    announce("tune_scene over the tiny scene")
    sc, choice = autotune.tune_scene("tiny-alpha", wl.vertices, rays, "alpha", cache_path=cache,
                                     leaf_sizes=(2, 4), steps=2, warmup=1, **ai)
    n_shapes = len(rtx.rt_launch_shapes())
    # f32 builds time every shape, compressed ones the default shape only,
    # packed ones the default shape and its variant without the queue,
    # four-wide ones the default shape and its 16-slot variant; each in index
    # and longest-path-first chunk order
    assert len(choice["ms"]) == 2 * 2 * (n_shapes + 1 + 2 + 2)
    # the close finalists of that pass are timed again, interleaved, and the
    # choice is the fastest of them
    label = (f"{choice['max_leaf']}/{choice['layout']}/{','.join(map(str, choice['shape']))}/"
             f"{'lf' if choice['longest_first'] else 'index'}")
    assert set(choice["finals_ms"]) <= set(choice["ms"]) and len(choice["finals_ms"]) <= 4
    if choice["finals_ms"]:
        assert min(choice["finals_ms"], key=choice["finals_ms"].get) == label
        first = min(choice["ms"], key=choice["ms"].get)
        assert first in choice["finals_ms"]
    else:
        assert min(choice["ms"], key=choice["ms"].get) == label
    # a queue shape's grid size is tuned next, over 4..8 waves per SIMD
    if choice["shape"][3]:
        assert sorted(choice["waves_ms"]) == ["4", "5", "6", "7", "8"]
        assert choice["waves_per_simd"] in (4, 5, 6, 7, 8)
    else:
        assert choice["waves_per_simd"] is None and choice["waves_ms"] == {}
    assert sc.info.max_leaf == choice["max_leaf"]
    assert sc.info.layout == rtx.LAYOUTS[choice["layout"]]
    hits, cnt = rtx.trace(sc, rays, "alpha", count=True, alpha_min=128,
                          shape=tuple(choice["shape"]), longest_first=choice["longest_first"],
                          waves_per_simd=choice["waves_per_simd"])
    torch.cuda.synchronize()
    bvh = oracle_lib.build_bvh(wl.vertices, max_leaf=choice["max_leaf"])
    B = oracle_lib.traverse(wl.vertices, bvh, wl.rays, "alpha", layout=choice["layout"],
                            alpha_min=128, **ai)
    P.assert_exact_vs_b(P.hits_to_numpy(hits), B, "tuned tiny")
    P.assert_counters_vs_b(cnt, B, "tuned tiny")
    _, again = autotune.tune_scene("tiny-alpha", wl.vertices, rays, "alpha", cache_path=cache,
                                   leaf_sizes=(2, 4), **ai)
    assert again == choice


def test_tune_scene_times_the_given_query(env, oracle_lib):
    """tune_scene with the any-hit and the multi-hit query (its output buffer
    sized for k hits): the chosen build's occluders equal oracle B's, and its
    k nearest hits equal those of the same scene in the default shape."""
    torch, rtx = env
    from paper_1912_12786_amd import autotune
    wl = W.tiny()
    ai = tiny_alpha_inputs(wl.n_tris)
    rays = torch.from_numpy(wl.rays).cuda()
    kw = dict(leaf_sizes=(2,), layouts=("f32", "f32p"), waves=(6, 7), steps=1, warmup=1,
              rounds=1, cache_path=None, **ai)
    announce("tune_scene with the any-hit query")
    sc, choice = autotune.tune_scene("tiny-any", wl.vertices, rays, "alpha", query="any", **kw)
    occ = rtx.trace(sc, rays, "alpha", query="any", alpha_min=128, shape=tuple(choice["shape"]),
                    longest_first=choice["longest_first"], waves_per_simd=choice["waves_per_simd"])
    torch.cuda.synchronize()
    bvh = oracle_lib.build_bvh(wl.vertices, max_leaf=choice["max_leaf"])
    B = oracle_lib.traverse(wl.vertices, bvh, wl.rays, "alpha", any_hit=True,
                            layout=choice["layout"], alpha_min=128, **ai)
    assert np.array_equal(P.occluders_to_numpy(occ), B["prim"])
    announce("tune_scene with the 3-nearest query")
    sc, choice = autotune.tune_scene("tiny-multi", wl.vertices, rays, "alpha", query="multi", k=3,
                                     **kw)
    got, n_got = rtx.trace(sc, rays, "alpha", query="multi", k=3, alpha_min=128,
                           shape=tuple(choice["shape"]), longest_first=choice["longest_first"],
                           waves_per_simd=choice["waves_per_simd"])
    ref, n_ref = rtx.trace(sc, rays, "alpha", query="multi", k=3, alpha_min=128)
    torch.cuda.synchronize()
    assert torch.equal(n_got, n_ref)
    assert torch.equal(got.view(torch.int32), ref.view(torch.int32))


@pytest.mark.parametrize("seed", range(8))
def test_random_builds_bit_exact(env, oracle_lib, seed):
    """The random sweep's scenes and rays with a random leaf size limit and
    node layout, every intersector and query, against oracle B built and
    laid out the same way."""
    from tests.test_gpu_random import random_case
    from tests.test_oracle_pins import _scene_params
    torch, rtx = env
    rng, verts, rays = random_case(200 + seed)
    max_leaf = int(rng.integers(1, 8))
    layout = ["f32", "q8", "f32p"][(seed + seed // 3) % 3]
    kind = ["default", "alpha", "procedural"][seed % 3]
    query = ["closest", "any", "multi"][(seed // 2) % 3]
    k = int(rng.integers(1, 9))
    kw = _scene_params(rng, kind, verts.shape[0])
    announce(f"random build seed={seed} tris={verts.shape[0]} rays={rays.shape[0]} "
             f"max_leaf={max_leaf} layout={layout} kind={kind} query={query} k={k}")
    sc = rtx.upload_scene(verts, kw.get("geom_ids"), kw.get("texcoords"), kw.get("textures"),
                          layout=layout, max_leaf=max_leaf)
    tkw = {kk: kw[kk] for kk in ("alpha_min", "checker_n") if kk in kw}
    res, cnt = rtx.trace(sc, torch.from_numpy(rays).cuda(), kind, query=query, k=k, count=True, **tkw)
    torch.cuda.synchronize()
    bvh = oracle_lib.build_bvh(verts, max_leaf=max_leaf)
    B = oracle_lib.traverse(verts, bvh, rays, kind, any_hit=(query == "any"),
                            multi_k=(k if query == "multi" else 0), layout=layout, **kw)
    P.assert_counters_vs_b(cnt, B, f"random build {seed}")
    if query == "closest":
        P.assert_exact_vs_b(P.hits_to_numpy(res), B, f"random build {seed}")
    elif query == "any":
        assert np.array_equal(P.occluders_to_numpy(res), B["prim"])
    else:
        hits, nh = res
        h = hits.cpu().numpy()
        assert np.array_equal(nh.cpu().numpy().view(np.uint32), B["n_hits"])
        assert np.array_equal(np.ascontiguousarray(h[..., 1]).view(np.uint32),
                              np.asarray(B["prim"], np.uint32).reshape(-1, k))
        for col, key in ((0, "t"), (2, "u"), (3, "v")):
            assert np.array_equal(h[..., col].view(np.uint32),
                                  np.ascontiguousarray(B[key], np.float32).reshape(-1, k).view(np.uint32))
