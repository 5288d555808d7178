"""A user-defined intersector (tests/custom/prim_mask.hip: keep a hit iff
mask[prim_id] != 0) compiled against the traversal template.

Its results equal, bit for bit and with all four counters, the built-in alpha
intersector on textures that encode the same decision (texture 0 fully
transparent, texture 1 fully opaque, geom_id = mask), which oracle B checks
exactly; and the closest kept hit is the float64 closest hit of the sub-scene
of kept triangles (oracle A on that sub-scene, outside its exception set)."""
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
    from tests.custom import binding
    rtx.load_library()
    binding.load()
    return torch, rtx, binding


def mask_textures():
    # texture 0: alpha 0 (reject); texture 1: alpha 255 (accept); 1x1 texels
    return np.array([[[0x00000000]], [[0xFF000000]]], np.uint32)


@pytest.mark.parametrize("workload", ["tiny", "billboards"])
def test_custom_mask_intersector(env, oracle_lib, workload):
    torch, rtx, binding = env
    wl = W.tiny() if workload == "tiny" else W.billboards()
    rng = np.random.default_rng(31)
    mask = (rng.uniform(size=wl.n_tris) < 0.6).astype(np.uint8)
    announce(f"custom per-primitive mask intersector, {wl.name}, {int(mask.sum())} kept")
    scene = rtx.upload_scene(wl.vertices)
    rays = torch.from_numpy(wl.rays).cuda()
    m = torch.from_numpy(mask).cuda()
    hits, cnt = binding.trace(scene, rays, m, count=True)
    plain = binding.trace(scene, rays, m)
    # the built-in alpha intersector making the same decision
    geom = mask.astype(np.uint32)
    tc = np.zeros((wl.n_tris, 3, 2), np.float32)
    tex = mask_textures()
    ascene = rtx.upload_scene(wl.vertices, geom, tc, tex)
    ah, ac = rtx.trace(ascene, rays, "alpha", alpha_min=128, count=True)
    torch.cuda.synchronize()
    assert torch.equal(hits.view(torch.int32), ah.view(torch.int32))
    assert torch.equal(cnt, ac)
    assert torch.equal(plain.view(torch.int32), hits.view(torch.int32))
    # oracle B with the same encoding, bit for bit
    bvh = oracle_lib.build_bvh(wl.vertices)
    idx = np.arange(wl.n_rays) if workload == "tiny" else np.arange(0, wl.n_rays, 7)
    B = oracle_lib.traverse(wl.vertices, bvh, wl.rays[idx], "alpha", geom_ids=geom, texcoords=tc,
                            textures=tex, alpha_min=128)
    g = P.hits_to_numpy(hits)
    P.assert_exact_vs_b({k: v[idx] for k, v in g.items()}, B, "custom mask")
    assert np.array_equal(cnt.cpu().numpy().view(np.uint32)[idx], B["counters"])
    # the definition: closest hit of the kept sub-scene
    keep = np.nonzero(mask)[0]
    sub = W.subsample_indices(wl.n_rays, None, None, seed=3, n_random=2048)
    A = oracle_lib.brute(wl.vertices[keep], wl.rays, "default", ray_index=sub)
    ok = A["flags"] == 0
    gp = g["prim"][sub]
    mapped = np.where(A["prim"] == MISS, MISS, keep[np.minimum(A["prim"], len(keep) - 1)])
    assert ok.mean() > 0.9
    assert np.array_equal(gp[ok], mapped[ok].astype(np.uint32))
    assert (gp != MISS).mean() > 0.1


# ----------------------------------------------------------------------------
# intersectors defined from Python (paper_1912_12786_amd.custom)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("workload", ["tiny", "billboards"])
def test_python_defined_checker_and_alpha_equal_builtins(env, workload):
    """A checker and an alpha mask written as user code and compiled into
    their own kernels give the built-in intersectors' hits and counters bit
    for bit (both layouts of the scene); oracle B pins the built-ins."""
    torch, rtx, _ = env
    from tests.custom import python_defined as PD
    wl = W.tiny() if workload == "tiny" else W.billboards()
    if workload == "tiny":
        rng = np.random.default_rng(5)
        geom = rng.integers(0, 4, size=wl.n_tris).astype(np.uint32)
        tc = rng.uniform(0, 1, size=(wl.n_tris, 3, 2)).astype(np.float32)
        tex = W.alpha_textures(4, 64, 6)
    else:
        geom, tc, tex = wl.geom_ids, wl.texcoords, wl.textures
    rays = torch.from_numpy(wl.rays).cuda()
    checker = PD.load("user_checker")
    alpha = PD.load("user_alpha")
    for layout in ("f32", "q8"):
        announce(f"python-defined checker and alpha, {wl.name}, {layout}")
        sc = rtx.upload_scene(wl.vertices, geom, tc, tex, layout=layout, max_leaf=2)
        h, c = checker.trace(sc, rays, checker.params(n=8.0), count=True)
        rh, rc = rtx.trace(sc, rays, "procedural", checker_n=8, count=True)
        ap = alpha.params(texcoords=sc.texcoords, textures=sc.textures, width=int(tex.shape[2]),
                          height=int(tex.shape[1]), alpha_min=128)
        ah, ac = alpha.trace(sc, rays, ap, count=True)
        plain = alpha.trace(sc, rays, ap)
        rah, rac = rtx.trace(sc, rays, "alpha", alpha_min=128, count=True)
        torch.cuda.synchronize()
        assert torch.equal(h.view(torch.int32), rh.view(torch.int32)) and torch.equal(c, rc)
        assert torch.equal(ah.view(torch.int32), rah.view(torch.int32)) and torch.equal(ac, rac)
        assert torch.equal(plain.view(torch.int32), ah.view(torch.int32))
        assert (c[:, 2] > c[:, 3]).any() and (ac[:, 2] > ac[:, 3]).any()   # both masks reject
        # the any-hit query (shadow rays through the masks)
        ao, aoc = alpha.trace(sc, rays, ap, query="any", count=True)
        rao, raoc = rtx.trace(sc, rays, "alpha", query="any", alpha_min=128, count=True)
        co = checker.trace(sc, rays, checker.params(n=8.0), query="any")
        rco = rtx.trace(sc, rays, "procedural", query="any", checker_n=8)
        torch.cuda.synchronize()
        assert torch.equal(ao, rao) and torch.equal(aoc, raoc) and torch.equal(co, rco)
        assert torch.equal(ao != -1, rah[:, 1].view(torch.int32) != -1)


def test_python_defined_wireframe(env, oracle_lib):
    """A wireframe mask (keep a hit iff its barycentric distance to an edge,
    min(u, v, 1-u-v), is below a width): every kept hit satisfies it, lies
    no nearer than the unfiltered closest hit, and at width 1 (every point
    qualifies) the results equal the accept-all intersector and oracle B; at
    width -1 nothing qualifies (not 0: (1 - u) - v may round below 0 on a
    candidate whose u + v passed the triangle test)."""
    torch, rtx, _ = env
    from tests.custom import python_defined as PD
    wl = W.billboards()
    rays = torch.from_numpy(wl.rays).cuda()
    wire = PD.load("wireframe")
    sc = rtx.upload_scene(wl.vertices, max_leaf=2)
    announce("python-defined wireframe mask, billboards")
    h, c = wire.trace(sc, rays, wire.params(width=0.05), count=True)
    d = rtx.trace(sc, rays, "default")
    all_, call = wire.trace(sc, rays, wire.params(width=1.0), count=True)
    dc = rtx.trace(sc, rays, "default", count=True)[1]
    none, cnone = wire.trace(sc, rays, wire.params(width=-1.0), count=True)
    torch.cuda.synchronize()
    g = P.hits_to_numpy(h)
    gd = P.hits_to_numpy(d)
    hit = g["prim"] != MISS
    # fewer rays hit than with the accept-all intersector (some see only quad interiors)
    assert 0.02 < hit.mean() < (gd["prim"] != MISS).mean()
    u, v = g["u"][hit], g["v"][hit]
    m = np.minimum(np.minimum(u, v), (np.float32(1) - u) - v)
    assert np.all(m < np.float32(0.05))
    assert np.all(gd["prim"][hit] != MISS) and np.all(g["t"][hit] >= gd["t"][hit])
    assert torch.equal(all_.view(torch.int32), d.view(torch.int32))
    assert torch.equal(call[:, :2], dc[:, :2])
    B = oracle_lib.traverse(wl.vertices, oracle_lib.build_bvh(wl.vertices, max_leaf=2), wl.rays[::13])
    P.assert_exact_vs_b({k: v[::13] for k, v in P.hits_to_numpy(all_).items()}, B, "wire width 1")
    assert np.all(P.hits_to_numpy(none)["prim"] == MISS)
    assert int(cnone[:, 3].sum()) == 0 and int(cnone[:, 2].sum()) > 0
