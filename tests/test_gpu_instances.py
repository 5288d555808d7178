"""GPU parity of the instanced (two-level) traversal against oracle B's
float32 two-level traversal (bit-exact hits, instance ids and counters) and
the float64 definition."""
import numpy as np
import pytest

from paper_1912_12786_amd import workloads as W
from tests import parity as P
from tests.golden.load import load
from tests.test_oracle_instances import _billboard_meshes, world_boxes

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


def aimed_rays(wl, n_inst, seed):
    rng = np.random.default_rng(seed)
    rays = wl["rays"].copy()
    k = rays.shape[0] // 2
    tgt = wl["world_from_object"][rng.integers(0, n_inst, size=k), :, 3]
    d = tgt - rays[:k, :3].astype(np.float64)
    rays[:k, 4:7] = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    return rays


def test_golden_instances_gpu(env):
    torch, rtx = env
    fx = load("instances.json")
    mesh = fx["vertices"]
    for case in fx["cases"]:
        announce(f"golden instances {case['maps']}")
        maps = np.asarray(case["maps"], np.float32)
        lo, hi = world_boxes(mesh, maps)
        sc = rtx.InstancedScene([mesh], np.zeros(len(maps), np.uint32), maps, lo, hi)
        hits, inst = sc.trace(torch.from_numpy(fx["rays"]).cuda())
        torch.cuda.synchronize()
        g = P.hits_to_numpy(hits)
        assert (int(inst.cpu()[0]), int(g["prim"][0])) == (case["inst"], case["prim"])
        assert (g["t"][0], g["u"][0], g["v"][0]) == (case["t"], case["u"], case["v"])


def test_golden_alpha_instances_gpu(env):
    """The alpha-mask fixture split over two instanced meshes: the hit lies in
    the second instance behind a rejected candidate of the first; counters
    as derived by hand for the oracle."""
    torch, rtx = env
    announce("golden alpha instances")
    fx, meshes, geoms, tcs, tex, maps = _billboard_meshes()
    ids = np.array([0, 1], np.uint32)
    lo = np.array([[-1, -1, 0], [-1, -1, -1]], np.float32) - 1e-3
    hi = np.array([[1, 1, 0], [1, 1, -1]], np.float32) + 1e-3
    sc = rtx.InstancedScene(meshes, ids, maps, lo, hi, geom_ids=geoms, texcoords=tcs, textures=tex)
    rays = torch.from_numpy(fx["rays"]).cuda()
    hits, inst, cnt = sc.trace(rays, "alpha", alpha_min=128, count=True)
    dh, dinst, dcnt = sc.trace(rays, "default", count=True)
    occ, oinst = sc.trace(rays, "alpha", any_hit=True)
    torch.cuda.synchronize()
    g = P.hits_to_numpy(hits)
    assert (int(inst.cpu()[0]), int(g["prim"][0])) == (1, 1)
    assert (g["t"][0], g["u"][0], g["v"][0]) == (2.0, 0.625, 0.0625)
    assert cnt.cpu()[0].tolist() == [3, 4, 2, 1]
    d = P.hits_to_numpy(dh)
    assert (int(dinst.cpu()[0]), int(d["prim"][0]), d["t"][0]) == (0, 1, 1.0)
    assert dcnt.cpu()[0].tolist() == [3, 2, 1, 1]
    assert (int(occ.cpu()[0]), int(oinst.cpu()[0])) == (1, 1)


def alpha_inputs(wl, seed):
    """Per-mesh texture ids and coordinates, one shared texture array."""
    rng = np.random.default_rng(seed)
    tex = W.alpha_textures(3, 64, seed)
    geoms = [rng.integers(0, 3, size=m.shape[0]).astype(np.uint32) for m in wl["blas"]]
    tcs = [rng.uniform(0, 1, size=(m.shape[0], 3, 2)).astype(np.float32) for m in wl["blas"]]
    return dict(geom_ids=geoms, texcoords=tcs, textures=tex)


@pytest.mark.parametrize("kind", ["default", "procedural", "alpha"])
@pytest.mark.parametrize("any_hit", [False, True])
def test_instanced_parity(env, oracle_lib, kind, any_hit):
    torch, rtx = env
    n_inst = 300
    wl = W.instanced(n_inst, 320, 180)
    rays = aimed_rays(wl, n_inst, 7)
    akw = alpha_inputs(wl, 41) if kind == "alpha" else {}
    announce(f"instanced {n_inst} instances kind={kind} any={any_hit} rays={rays.shape[0]}")
    sc = rtx.InstancedScene(wl["blas"], wl["inst_blas"], wl["inst_m"], wl["world_lo"], wl["world_hi"],
                            **akw)
    out, inst, cnt = sc.trace(torch.from_numpy(rays).cuda(), kind, any_hit=any_hit, count=True)
    torch.cuda.synchronize()
    bvhs = [oracle_lib.build_bvh(b) for b in wl["blas"]]
    tl = oracle_lib.build_tlas(wl["world_lo"], wl["world_hi"])
    B = oracle_lib.traverse_instanced(wl["blas"], bvhs, wl["inst_blas"], wl["inst_m"], tl, rays,
                                      kind, any_hit=any_hit, **akw)
    if kind == "alpha":  # the mask rejects candidates on this workload
        assert (B["counters"][:, 2] > B["counters"][:, 3]).sum() > 100
    gi = inst.cpu().numpy().view(np.uint32)
    assert np.array_equal(gi, B["inst"])
    P.assert_counters_vs_b(cnt, B, f"instanced {kind} any={any_hit}")
    if any_hit:
        assert np.array_equal(out.cpu().numpy().view(np.uint32), B["prim"])
        return
    g = P.hits_to_numpy(out)
    P.assert_exact_vs_b(g, B, f"instanced {kind}")
    assert (g["prim"] != MISS).mean() > 0.2
    idx = np.arange(0, rays.shape[0], 97)
    A = oracle_lib.brute_instanced(wl["blas"], wl["inst_blas"], wl["inst_m"], rays[idx], kind, **akw)
    ok = A["flags"] == 0
    assert np.array_equal(g["prim"][idx][ok], A["prim"][ok])
    assert np.array_equal(gi[idx][ok], A["inst"][ok])


def test_identity_instance_equals_plain_trace(env):
    torch, rtx = env
    wl = W.tiny()
    announce("identity instance of the tiny scene")
    maps = np.array([[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]], np.float32)
    lo, hi = world_boxes(wl.vertices, maps)
    isc = rtx.InstancedScene([wl.vertices], np.zeros(1, np.uint32), maps, lo, hi)
    rays = torch.from_numpy(wl.rays).cuda()
    hits, inst = isc.trace(rays)
    plain = rtx.trace(rtx.upload_scene(wl.vertices), rays)
    torch.cuda.synchronize()
    assert torch.equal(hits.view(torch.int32), plain.view(torch.int32))


@pytest.mark.parametrize("kind", ["default", "alpha"])
def test_instanced_bench_config_sampled(env, oracle_lib, kind):
    """The benchmark's instanced launch (2,000 instances, 1920x1080 rays, one
    call over all rays) against oracle B's two-level traversal on every 61st
    ray: hits, instance ids and counters bit for bit."""
    torch, rtx = env
    wl = W.instanced(2000)
    akw = W.instanced_alpha(wl) if kind == "alpha" else {}
    announce(f"instanced bench config kind={kind} rays={wl['rays'].shape[0]}")
    sc = rtx.InstancedScene(wl["blas"], wl["inst_blas"], wl["inst_m"], wl["world_lo"], wl["world_hi"],
                            **akw)
    rays = wl["rays"]
    out, inst, cnt = sc.trace(torch.from_numpy(rays).cuda(), kind, count=True)
    plain, plain_inst = sc.trace(torch.from_numpy(rays).cuda(), kind)
    torch.cuda.synchronize()
    # the counting launch and the timed (non-counting) launch agree everywhere
    assert torch.equal(out.view(torch.int32), plain.view(torch.int32))
    assert torch.equal(inst, plain_inst)
    idx = np.arange(5, rays.shape[0], 61)
    bvhs = [oracle_lib.build_bvh(b) for b in wl["blas"]]
    tl = oracle_lib.build_tlas(wl["world_lo"], wl["world_hi"])
    B = oracle_lib.traverse_instanced(wl["blas"], bvhs, wl["inst_blas"], wl["inst_m"], tl, rays[idx],
                                      kind, **akw)
    g = P.hits_to_numpy(out[torch.from_numpy(idx).cuda()])
    P.assert_exact_vs_b(g, B, f"instanced bench config {kind}")
    assert np.array_equal(inst.cpu().numpy().view(np.uint32)[idx], B["inst"])
    P.assert_counters_vs_b(cnt[torch.from_numpy(idx).cuda()], B, f"instanced bench config {kind}")
    assert (g["prim"] != MISS).mean() > 0.05
    if kind == "alpha":
        assert (B["counters"][:, 2] > B["counters"][:, 3]).sum() > 100
