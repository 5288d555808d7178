"""Seeded random instanced scenes on the GPU against oracle B's two-level
traversal, bit for bit (hits, instance ids, counters): several meshes,
duplicated instances (exact ties between instances), mirrored and strongly
scaled maps, empty meshes, rays aimed at instances and stray rays; the three
built-in masks (alpha with per-mesh texture ids and coordinates)."""
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


def random_instances(seed):
    rng = np.random.default_rng(5000 + seed)
    meshes = []
    for b in range(int(rng.integers(1, 5))):
        n = int(rng.integers(0, 400)) if b else int(rng.integers(1, 400))
        meshes.append(W.random_triangles(n, 7000 + 10 * seed + b, side=0.4, box=(-1.0, 1.0))
                      if n else np.zeros((0, 3, 3), np.float32))
    n_inst = int(rng.integers(1, 200))
    ids = rng.integers(0, len(meshes), size=n_inst).astype(np.uint32)
    wfo = np.empty((n_inst, 3, 4))
    for q in range(n_inst):
        L = W._rotation(rng) * rng.uniform(0.05, 4.0)
        if rng.integers(0, 4) == 0:
            L[:, 0] *= -1.0                                   # mirrored
        wfo[q, :, :3] = L
        wfo[q, :, 3] = rng.uniform(0, 20, size=3)
    dup = rng.integers(0, n_inst, size=n_inst // 5)
    if n_inst > 1 and dup.size:                               # identical instances
        wfo[dup] = wfo[(dup + 1) % n_inst]
        ids[dup] = ids[(dup + 1) % n_inst]
    lo = np.stack([m.reshape(-1, 3).min(0) if m.size else np.zeros(3) for m in meshes])[ids]
    hi = np.stack([m.reshape(-1, 3).max(0) if m.size else np.zeros(3) for m in meshes])[ids]
    maps, wlo, whi = W.instance_transforms(wfo, lo.astype(np.float64), hi.astype(np.float64))
    m = int(rng.integers(1, 3000))
    o = rng.uniform(-5, 25, size=(m, 3))
    tgt = np.where(rng.uniform(size=(m, 1)) < 0.7, wfo[rng.integers(0, n_inst, size=m), :, 3],
                   rng.uniform(0, 20, size=(m, 3)))
    d = tgt - o
    d /= np.maximum(np.linalg.norm(d, axis=1, keepdims=True), 1e-12)
    rays = np.zeros((m, 8), np.float32)
    rays[:, :3] = o
    rays[:, 4:7] = d
    rays[:, 7] = np.inf
    return meshes, ids, maps, wlo, whi, rays


@pytest.mark.parametrize("seed", range(8))
def test_random_instanced_bit_exact(env, oracle_lib, seed):
    torch, rtx = env
    meshes, ids, maps, lo, hi, rays = random_instances(seed)
    kind = ["default", "procedural", "alpha"][seed % 3]
    any_hit = bool((seed // 3) % 2)
    akw = {}
    if kind == "alpha":
        rng = np.random.default_rng(6000 + seed)
        n_tex = int(rng.integers(1, 5))
        akw = dict(geom_ids=[rng.integers(0, n_tex, size=m.shape[0]).astype(np.uint32)
                             for m in meshes],
                   texcoords=[rng.uniform(-0.2, 1.2, size=(m.shape[0], 3, 2)).astype(np.float32)
                              for m in meshes],
                   textures=W.alpha_textures(n_tex, int(rng.integers(16, 65)), 6100 + seed))
    announce(f"random instanced seed={seed} meshes={len(meshes)} instances={len(ids)} "
             f"rays={rays.shape[0]} kind={kind} any={any_hit}")
    sc = rtx.InstancedScene(meshes, ids, maps, lo, hi, **akw)
    out, inst, cnt = sc.trace(torch.from_numpy(rays).cuda(), kind, any_hit=any_hit, count=True)
    torch.cuda.synchronize()
    bvhs = [oracle_lib.build_bvh(b) for b in meshes]
    tl = oracle_lib.build_tlas(lo, hi)
    B = oracle_lib.traverse_instanced(meshes, bvhs, ids, maps, tl, rays, kind, any_hit=any_hit, **akw)
    P.assert_counters_vs_b(cnt, B, f"random instanced {seed}")
    assert np.array_equal(inst.cpu().numpy().view(np.uint32), B["inst"])
    if any_hit:
        assert np.array_equal(out.cpu().numpy().view(np.uint32), B["prim"])
    else:
        P.assert_exact_vs_b(P.hits_to_numpy(out), B, f"random instanced {seed}")
