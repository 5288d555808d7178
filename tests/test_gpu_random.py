"""Seeded random sweep on the GPU against oracle B, bit for bit (hits,
occluders, multi-hit lists and all four counters): scenes with duplicated
triangles (exact ties), zero-area and sliver triangles, clustered and spread
geometry; rays with zero, tiny and axis-aligned direction components, finite
intervals and origins inside the scene; every intersector, query and compiled
launch shape, with ragged ray counts."""
import numpy as np
import pytest

from tests import parity as P
from tests.test_oracle_pins import _scene_params

pytestmark = pytest.mark.gpu
MISS = 0xFFFFFFFF
SEEDS = range(16)


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1912_12786_amd import rtx
    rtx.load_library()
    return torch, rtx


def random_case(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 3000))
    clusters = rng.uniform(0, 10, size=(int(rng.integers(1, 6)), 3))
    c = clusters[rng.integers(0, len(clusters), size=n)] + rng.normal(0, 1, size=(n, 3))
    s = rng.uniform(0.02, 0.8, size=(n, 1, 1))
    v = c[:, None, :] + s * rng.normal(0, 1, size=(n, 3, 3))
    kinds = rng.integers(0, 6, size=n)
    v[kinds == 1, 2] = v[kinds == 1, 1]                              # zero area
    v[kinds == 2, 2] = v[kinds == 2, 0] + 1e-4 * (v[kinds == 2, 1] - v[kinds == 2, 0])  # sliver
    dup = np.nonzero(kinds == 3)[0]
    if dup.size and n > 1:                                           # exact duplicates
        v[dup] = v[rng.integers(0, n, size=dup.size)]
    v = v.astype(np.float32)
    m = int(rng.integers(1, 5000))
    o = rng.uniform(-3, 13, size=(m, 3))
    tgt = rng.uniform(0, 10, size=(m, 3))
    d = tgt - o
    d /= np.maximum(np.linalg.norm(d, axis=1, keepdims=True), 1e-12)
    mode = rng.integers(0, 8, size=m)
    axis = rng.integers(0, 3, size=m)
    d[mode == 1, axis[mode == 1]] = 0.0
    d[mode == 2, axis[mode == 2]] = 1e-30
    ax = mode == 3
    d[ax] = 0.0
    d[ax, axis[ax]] = rng.choice([-1.0, 1.0], size=int(ax.sum()))
    rays = np.zeros((m, 8), np.float32)
    rays[:, :3] = o
    rays[:, 4:7] = d
    rays[:, 7] = np.inf
    fin = mode == 4
    rays[fin, 3] = rng.uniform(0, 3, size=int(fin.sum()))
    rays[fin, 7] = rays[fin, 3] + rng.uniform(0, 10, size=int(fin.sum()))
    return rng, v, rays


@pytest.mark.parametrize("seed", SEEDS)
def test_random_scene_bit_exact(env, oracle_lib, seed):
    torch, rtx = env
    rng, verts, rays = random_case(seed)
    kind = ["default", "alpha", "procedural"][seed % 3]
    query = ["closest", "any", "multi"][(seed // 3) % 3]
    k = int(rng.integers(1, 9))
    shapes = rtx.rt_launch_shapes()
    shape = shapes[seed % len(shapes)]
    kw = _scene_params(rng, kind, verts.shape[0])
    announce(f"random seed={seed} tris={verts.shape[0]} rays={rays.shape[0]} kind={kind} "
             f"query={query} k={k} shape={shape}")
    sc = rtx.upload_scene(verts, kw.get("geom_ids"), kw.get("texcoords"), kw.get("textures"))
    tkw = {kk: kw[kk] for kk in ("alpha_min", "checker_n") if kk in kw}
    bvh = oracle_lib.build_bvh(verts)
    out = rtx.trace(sc, torch.from_numpy(rays).cuda(), kind, query=query, k=k, count=True,
                    shape=shape, **tkw)
    torch.cuda.synchronize()
    res, cnt = out
    B = oracle_lib.traverse(verts, bvh, rays, kind, any_hit=(query == "any"),
                            multi_k=(k if query == "multi" else 0), **kw)
    P.assert_counters_vs_b(cnt, B, f"random {seed}")
    if query == "closest":
        P.assert_exact_vs_b(P.hits_to_numpy(res), B, f"random {seed}")
    elif query == "any":
        assert np.array_equal(P.occluders_to_numpy(res), B["prim"])
    else:
        hits, nh = res
        h = hits.cpu().numpy()
        assert np.array_equal(nh.cpu().numpy().view(np.uint32), B["n_hits"])
        gp = np.ascontiguousarray(h[..., 1]).view(np.uint32)
        bp = np.asarray(B["prim"], np.uint32).reshape(-1, k)
        bad = np.nonzero(np.any(gp != bp, axis=1))[0]
        assert bad.size == 0, (f"{bad.size} rays differ, first {bad[:4]}: gpu {gp[bad[:2]].tolist()} "
                               f"oracle {bp[bad[:2]].tolist()} t gpu {h[bad[:2], :, 0].tolist()} "
                               f"oracle {np.asarray(B['t']).reshape(-1, k)[bad[:2]].tolist()} "
                               f"rays {rays[bad[:2]].tolist()}")
        for col, key in ((0, "t"), (2, "u"), (3, "v")):
            assert np.array_equal(h[..., col].view(np.uint32),
                                  np.ascontiguousarray(B[key], np.float32).reshape(-1, k).view(np.uint32))
