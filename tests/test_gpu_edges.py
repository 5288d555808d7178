"""Edge cases of the widened entry points on the GPU: batches with empty
scenes, scenes without rays and single-leaf scenes; instanced scenes without
instances, with empty meshes and mirrored maps; multi-hit and backward on
single rays and all-miss rays.  Every result is checked against oracle B (or
against a fact that holds by construction)."""
import numpy as np
import pytest

from paper_1912_12786_amd import workloads as W
from tests import parity as P
from tests.test_oracle_instances import world_boxes

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


def test_batch_with_empty_and_tiny_scenes(env, oracle_lib):
    torch, rtx = env
    base = W.batched(4, tri_range=(2_000, 5_000), ray_range=(300, 700))
    tiny = W.tiny()
    scenes = [
        base[0],
        {"vertices": base[1]["vertices"], "rays": base[1]["rays"][:0]},        # no rays
        {"vertices": np.zeros((0, 3, 3), np.float32), "rays": tiny.rays[:77]},  # no triangles
        {"vertices": tiny.vertices[:3], "rays": tiny.rays[:129]},               # root is a leaf
        base[2],
        {"vertices": tiny.vertices, "rays": tiny.rays[:1]},                     # one ray
        base[3],
    ]
    n = [s["rays"].shape[0] for s in scenes]
    announce(f"batch with empty / single-leaf scenes, ray counts {n}")
    sc_list = [rtx.upload_scene(s["vertices"]) for s in scenes]
    batch = rtx.Batch(sc_list, n, "default")
    rays = torch.from_numpy(np.concatenate([s["rays"] for s in scenes])).cuda()
    hits, cnt = batch.trace(rays, count=True)
    torch.cuda.synchronize()
    g = P.hits_to_numpy(hits)
    c = cnt.cpu().numpy().view(np.uint32)
    off = batch.offsets
    for i, s in enumerate(scenes):
        sl = slice(off[i], off[i + 1])
        if n[i] == 0:
            continue
        bvh = oracle_lib.build_bvh(s["vertices"])
        B = oracle_lib.traverse(s["vertices"], bvh, s["rays"], "default")
        P.assert_exact_vs_b({k: v[sl] for k, v in g.items()}, B, f"edge batch scene {i}")
        assert np.array_equal(c[sl], B["counters"]), i
    assert np.all(g["prim"][off[2]:off[3]] == MISS)


def test_instanced_without_instances(env, oracle_lib):
    torch, rtx = env
    wl = W.instanced(10, 40, 30)
    announce("instanced scene with no instances")
    z = np.zeros((0, 3), np.float32)
    sc = rtx.InstancedScene(wl["blas"], np.zeros(0, np.uint32), np.zeros((0, 12), np.float32), z, z)
    out, inst, cnt = sc.trace(torch.from_numpy(wl["rays"]).cuda(), count=True)
    torch.cuda.synchronize()
    g = P.hits_to_numpy(out)
    assert np.all(g["prim"] == MISS) and np.all(inst.cpu().numpy().view(np.uint32) == MISS)
    assert np.all(cnt.cpu().numpy() == 0)


@pytest.mark.parametrize("n_rays", [1, 65, 1200])
def test_instanced_empty_mesh_and_mirrored_maps(env, oracle_lib, n_rays):
    torch, rtx = env
    n_inst = 60
    wl = W.instanced(n_inst, 40, 30)
    blas = wl["blas"] + [np.zeros((0, 3, 3), np.float32)]
    ids = wl["inst_blas"].copy()
    ids[::7] = 3                                  # some instances of an empty mesh
    wfo = wl["world_from_object"].copy()
    wfo[1::4, 0, :3] *= -1.0                      # mirrored instances (det < 0)
    blo = np.stack([b.reshape(-1, 3).min(0) if b.size else np.zeros(3) for b in blas])[ids]
    bhi = np.stack([b.reshape(-1, 3).max(0) if b.size else np.zeros(3) for b in blas])[ids]
    m, lo, hi = W.instance_transforms(wfo, blo.astype(np.float64), bhi.astype(np.float64))
    rng = np.random.default_rng(n_rays)
    rays = wl["rays"][rng.choice(wl["rays"].shape[0], size=n_rays, replace=False)].copy()
    k = n_rays // 2
    tgt = wfo[rng.integers(0, n_inst, size=k), :, 3]
    d = tgt - rays[:k, :3].astype(np.float64)
    rays[:k, 4:7] = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    announce(f"instanced: empty mesh, mirrored maps, {n_rays} rays")
    sc = rtx.InstancedScene(blas, ids, m, lo, hi)
    out, inst, cnt = sc.trace(torch.from_numpy(rays).cuda(), count=True)
    torch.cuda.synchronize()
    bvhs = [oracle_lib.build_bvh(b) for b in blas]
    tl = oracle_lib.build_tlas(lo, hi)
    B = oracle_lib.traverse_instanced(blas, bvhs, ids, m, tl, rays)
    P.assert_exact_vs_b(P.hits_to_numpy(out), B, "instanced edge")
    P.assert_counters_vs_b(cnt, B, "instanced edge")
    assert np.array_equal(inst.cpu().numpy().view(np.uint32), B["inst"])
    hit_inst = B["inst"][B["prim"] != MISS]
    assert not np.any(ids[hit_inst] == 3)


def test_multi_single_ray_and_all_miss(env, oracle_lib):
    torch, rtx = env
    wl = W.tiny()
    sc = rtx.upload_scene(wl.vertices)
    bvh = oracle_lib.build_bvh(wl.vertices)
    announce("multi-hit k=8 on one ray and on rays that miss everything")
    allB = oracle_lib.traverse(wl.vertices, bvh, wl.rays, "default", multi_k=8, count=False)
    best = int(np.argmax(allB["n_hits"]))       # the ray with the most hits
    centre = wl.rays[best:best + 1].copy()
    away = wl.rays[:100].copy()
    away[:, 4:7] *= -1.0                          # looking away from the scene
    for rays in (centre, away):
        hits, nh = rtx.trace(sc, torch.from_numpy(rays).cuda(), "default", query="multi", k=8)
        torch.cuda.synchronize()
        B = oracle_lib.traverse(wl.vertices, bvh, rays, "default", multi_k=8, count=False)
        h = hits.cpu().numpy().reshape(rays.shape[0], 8, 4)
        assert np.array_equal(nh.cpu().numpy().view(np.uint32), B["n_hits"])
        assert np.array_equal(h[..., 1].view(np.uint32), B["prim"].reshape(-1, 8))
        assert np.array_equal(h[..., 0].view(np.uint32), B["t"].reshape(-1, 8).view(np.uint32))
    assert np.all(B["n_hits"] == 0)


def test_backward_all_miss_and_empty(env):
    torch, rtx = env
    from paper_1912_12786_amd import diff
    wl = W.diff_scene(freq=10, n_billboards=10, width=16, height=16)
    announce("backward with all rays missing, and with no rays")
    rays = torch.from_numpy(wl.rays.copy()).cuda()
    rays[:, 4:7] *= -1.0                          # away from the sphere
    V = torch.from_numpy(wl.vertices).cuda()
    F = torch.from_numpy(wl.faces.astype(np.int32)).cuda()
    sc = rtx.upload_scene(wl.vertices[wl.faces])
    hits = rtx.trace(sc, rays, "default")
    assert torch.all(hits[:, 1].view(torch.int32) == -1)
    g = torch.ones((rays.shape[0], 3), device="cuda")
    gV, gR = diff.hit_backward(rays, hits, g, V, F)
    torch.cuda.synchronize()
    assert torch.all(gV == 0) and torch.all(gR == 0)
    gV0, gR0 = diff.hit_backward(rays[:0], hits[:0], g[:0], V, F)
    torch.cuda.synchronize()
    assert torch.all(gV0 == 0) and gR0.shape == (0, 8)
