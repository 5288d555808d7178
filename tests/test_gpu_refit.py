"""GPU parity of the device refit (rt_bvh_refit: a built tree's triangle
records and boxes recomputed from moved vertices, topology kept) against
oracle B's refit of its own tree, bit for bit, and of traversals of the
refitted tree against oracle B; the autograd forward with a refit scene.
The refit is not in the paper, whose BVH construction is open."""
import numpy as np
import pytest

from paper_1912_12786_amd import workloads as W
from tests import parity as P
from tests.test_capi_cpu import decode_oracle_bvh, decode_product_bvh

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


@pytest.fixture(scope="module")
def mesh():
    return W.diff_scene()


def download(rs):
    sc = rs.scene
    nodes = sc.nodes.cpu().numpy() if sc.nodes is not None else np.zeros(0, np.uint8)
    return nodes, sc.tris.cpu().numpy()


def assert_tree_equals_oracle(rs, obvh, soup):
    """Decoded product tree (root box from the refit) against the oracle's
    refitted tree, bounds bit for bit; triangle records from the moved mesh."""
    nodes, tris = download(rs)
    prod = decode_product_bvh(nodes, tris, rs.scene.info)
    orc = decode_oracle_bvh(obvh)
    assert len(prod) == len(orc)
    for a, b in zip(prod, orc):
        assert np.array_equal(np.array(a[0], np.float32).view(np.uint32),
                              np.array(b[0], np.float32).view(np.uint32))
        assert np.array_equal(np.array(a[1], np.float32).view(np.uint32),
                              np.array(b[1], np.float32).view(np.uint32))
        assert a[2:] == b[2:]
    tf = tris.view(np.float32).reshape(-1, 12)
    tu = tris.view(np.uint32).reshape(-1, 12)
    v = soup[obvh.perm]
    assert np.array_equal(tu[:, 3], obvh.perm)
    assert np.array_equal(tf[:, 0:3].view(np.uint32), v[:, 0].view(np.uint32))
    assert np.array_equal(tf[:, 4:7].view(np.uint32), (v[:, 1] - v[:, 0]).view(np.uint32))
    assert np.array_equal(tf[:, 8:11].view(np.uint32), (v[:, 2] - v[:, 0]).view(np.uint32))


def test_refit_to_build_vertices_is_identity(env, mesh):
    torch, rtx = env
    rs = rtx.RefitScene(mesh.vertices, mesh.faces, mesh.geom_ids, mesh.texcoords, mesh.textures,
                        max_leaf=2)
    before = download(rs)
    lo, hi = list(rs.scene.info.root_lo), list(rs.scene.info.root_hi)
    announce("refit of the diff scene to its own vertices")
    rs.update(torch.from_numpy(mesh.vertices).cuda())
    torch.cuda.synchronize()
    after = download(rs)
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    assert list(rs.scene.info.root_lo) == lo and list(rs.scene.info.root_hi) == hi


@pytest.mark.parametrize("sigma,max_leaf", [(0.003, 2), (0.05, 4), (0.3, 1), (0.01, 7)])
def test_refit_moved_matches_oracle(env, oracle_lib, mesh, sigma, max_leaf):
    """Moved vertices (the second of two refits in a row): the refitted tree
    equals oracle B's refit bit for bit, and alpha closest and any-hit
    traversals of it equal oracle B's on the moved mesh (hits, occluders,
    counters)."""
    torch, rtx = env
    rng = np.random.default_rng(int(sigma * 1000) + max_leaf)
    moved = (mesh.vertices + rng.normal(0.0, sigma, size=mesh.vertices.shape)).astype(np.float32)
    rs = rtx.RefitScene(mesh.vertices, mesh.faces, mesh.geom_ids, mesh.texcoords, mesh.textures,
                        max_leaf=max_leaf)
    announce(f"refit diff scene sigma={sigma} max_leaf={max_leaf} (after a first refit)")
    first = (mesh.vertices + rng.normal(0.0, 2 * sigma, size=mesh.vertices.shape)
             ).astype(np.float32)
    rs.update(torch.from_numpy(first).cuda())     # the counters must start from zero again
    rs.update(torch.from_numpy(moved).cuda())
    torch.cuda.synchronize()
    ob = oracle_lib.refit(oracle_lib.build_bvh(mesh.triangles, max_leaf=max_leaf), moved,
                          mesh.faces)
    soup = moved[mesh.faces]
    assert_tree_equals_oracle(rs, ob, soup)
    okw = dict(geom_ids=mesh.geom_ids, texcoords=mesh.texcoords, textures=mesh.textures,
               alpha_min=128)
    rays = torch.from_numpy(mesh.rays).cuda()
    hits, cnt = rtx.trace(rs.scene, rays, "alpha", count=True, alpha_min=128)
    occ, acnt = rtx.trace(rs.scene, rays, "alpha", query="any", count=True, alpha_min=128)
    torch.cuda.synchronize()
    B = oracle_lib.traverse(soup, ob, mesh.rays, "alpha", **okw)
    P.assert_exact_vs_b(P.hits_to_numpy(hits), B, f"refit sigma={sigma}")
    P.assert_counters_vs_b(cnt, B, f"refit sigma={sigma}")
    Ba = oracle_lib.traverse(soup, ob, mesh.rays, "alpha", any_hit=True, **okw)
    assert np.array_equal(P.occluders_to_numpy(occ), Ba["prim"])
    P.assert_counters_vs_b(acnt, Ba, f"refit any sigma={sigma}")
    assert (B["prim"] != MISS).mean() > 0.05


def oracle_slots(ob):
    """Oracle B's tree as the 64-byte nodes' child slots: for each inner node
    in preorder (the library's numbering), lo, hi of its first child then of
    its second, float32 [n_inner, 12]."""
    nd = ob.nodes
    inner = np.nonzero(nd["count"] == 0)[0]
    L, R = nd["left"][inner], nd["right"][inner]
    return np.concatenate([nd["lo"][L], nd["hi"][L], nd["lo"][R], nd["hi"][R]], axis=1)


@pytest.mark.parametrize("scene,max_leaf,top_range", [
    ("billboards", 1, (1025, 2048)),   # the top block's on-chip version, near full
    ("spheres", 2, (2049, 1 << 30)),   # more than it holds: the global version
])
def test_refit_long_top_lists(env, oracle_lib, scene, max_leaf, top_range):
    """Large trees whose top lists take each version of the top block (the
    on-chip one holds 2,048 nodes): every child slot, every triangle record
    and the root box bit for bit against oracle B's refit of its own build,
    after two refits in a row."""
    torch, rtx = env
    wl = W.billboards() if scene == "billboards" else W.spheres()
    v = wl.vertices.reshape(-1, 3).copy()
    f = np.arange(v.shape[0], dtype=np.uint32).reshape(-1, 3)
    rs = rtx.RefitScene(v, f, max_leaf=max_leaf)
    assert top_range[0] <= rs.n_top <= top_range[1]
    rng = np.random.default_rng(11)
    scale = float(np.abs(v).max())
    first = (v + rng.normal(0.0, 1e-3 * scale, size=v.shape)).astype(np.float32)
    moved = (v + rng.normal(0.0, 3e-4 * scale, size=v.shape)).astype(np.float32)
    announce(f"refit {scene} max_leaf={max_leaf}: {rs.scene.info.n_nodes} nodes, "
             f"{rs.n_top} top nodes")
    rs.update(torch.from_numpy(first).cuda())
    rs.update(torch.from_numpy(moved).cuda())
    torch.cuda.synchronize()
    ob = oracle_lib.refit(oracle_lib.build_bvh(wl.vertices, max_leaf=max_leaf), moved, f)
    nodes, tris = download(rs)
    got = nodes.view(np.uint32).reshape(-1, 16)[:, :12]
    assert np.array_equal(got, oracle_slots(ob).view(np.uint32))
    assert np.array_equal(np.array(rs.scene.info.root_lo[:], np.float32).view(np.uint32),
                          ob.nodes["lo"][0].view(np.uint32))
    assert np.array_equal(np.array(rs.scene.info.root_hi[:], np.float32).view(np.uint32),
                          ob.nodes["hi"][0].view(np.uint32))
    tf = tris.view(np.float32).reshape(-1, 12)
    tu = tris.view(np.uint32).reshape(-1, 12)
    sv = moved[f][ob.perm]
    assert np.array_equal(tu[:, 3], ob.perm)
    assert np.array_equal(tf[:, 0:3].view(np.uint32), sv[:, 0].view(np.uint32))
    assert np.array_equal(tf[:, 4:7].view(np.uint32), (sv[:, 1] - sv[:, 0]).view(np.uint32))
    assert np.array_equal(tf[:, 8:11].view(np.uint32), (sv[:, 2] - sv[:, 0]).view(np.uint32))


def test_refit_invalid_indices_and_root_leaf(env, oracle_lib):
    """Face indices past the vertices (written into the device faces) read
    NaN: boxes ignore those corners and their triangles are never hit, as in
    oracle B; a root leaf gets its root box from its triangles."""
    torch, rtx = env
    rng = np.random.default_rng(5)
    tiny = W.tiny()
    v = tiny.vertices.reshape(-1, 3).copy()
    f = np.arange(v.shape[0], dtype=np.uint32).reshape(-1, 3)
    rs = rtx.RefitScene(v, f, max_leaf=2)
    bad = f.copy()
    pick = rng.choice(f.shape[0], 40, replace=False)
    bad[pick, rng.integers(0, 3, 40)] = v.shape[0] + 7
    rs.faces.copy_(torch.from_numpy(bad.astype(np.int32)).cuda())
    moved = (v + rng.normal(0.0, 0.01, size=v.shape)).astype(np.float32)
    announce("refit with 40 out-of-range corners")
    rs.update(torch.from_numpy(moved).cuda())
    hits, cnt = rtx.trace(rs.scene, torch.from_numpy(tiny.rays).cuda(), count=True)
    torch.cuda.synchronize()
    ob = oracle_lib.refit(oracle_lib.build_bvh(tiny.vertices, max_leaf=2), moved, bad)
    vv = np.concatenate([moved, np.full((8, 3), np.nan, np.float32)])
    soup = vv[bad]
    nodes, tris = download(rs)
    prod = decode_product_bvh(nodes, tris, rs.scene.info)
    orc = decode_oracle_bvh(ob)
    for a, b in zip(prod, orc):
        assert np.array_equal(np.array(a[0], np.float32).view(np.uint32),
                              np.array(b[0], np.float32).view(np.uint32))
        assert np.array_equal(np.array(a[1], np.float32).view(np.uint32),
                              np.array(b[1], np.float32).view(np.uint32))
    B = oracle_lib.traverse(soup, ob, tiny.rays)
    g = P.hits_to_numpy(hits)
    P.assert_exact_vs_b(g, B, "refit invalid corners")
    P.assert_counters_vs_b(cnt, B, "refit invalid corners")
    assert not np.isin(g["prim"], pick).any()
    # a root leaf
    v3 = tiny.vertices[:3].reshape(-1, 3).copy()
    f3 = np.arange(9, dtype=np.uint32).reshape(3, 3)
    rl = rtx.RefitScene(v3, f3, max_leaf=4)
    assert rl.scene.info.n_nodes == 0
    m3 = (v3 + 0.5).astype(np.float32)
    announce("refit of a root leaf")
    rl.update(torch.from_numpy(m3).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(np.array(rl.scene.info.root_lo[:], np.float32), m3.min(0))
    assert np.array_equal(np.array(rl.scene.info.root_hi[:], np.float32), m3.max(0))


def test_autograd_with_refit(env, mesh):
    """The autograd forward with a refit scene: at the build's vertices the
    same bits as the rebuilding forward; after a move, the hits of a fresh
    trace of the refitted tree, and finite gradients."""
    import torch
    from paper_1912_12786_amd import diff
    _, rtx = env
    rs = rtx.RefitScene(mesh.vertices, mesh.faces, mesh.geom_ids, mesh.texcoords, mesh.textures,
                        max_leaf=2)
    rays = torch.from_numpy(mesh.rays).cuda()
    F = torch.from_numpy(mesh.faces.astype(np.int32)).cuda()
    V = torch.from_numpy(mesh.vertices).cuda()
    announce("DifferentiableHit with a refit scene")
    ref = diff.DifferentiableHit.apply(rays, V, F, mesh.geom_ids, mesh.texcoords, mesh.textures,
                                       "alpha", 128, 8, 2, 512)
    got = diff.DifferentiableHit.apply(rays, V, F, None, None, None, "alpha", 128, 8, 2, 512, rs)
    torch.cuda.synchronize()
    assert torch.equal(ref[0].view(torch.int32), got[0].view(torch.int32))
    assert torch.equal(ref[1], got[1])
    moved = (V + 0.01 * torch.randn(V.shape, generator=torch.Generator("cuda").manual_seed(3),
                                    device="cuda")).requires_grad_(True)
    r2 = rays.clone().requires_grad_(True)
    tuv, prim, hit = diff.DifferentiableHit.apply(r2, moved, F, None, None, None, "alpha", 128, 8,
                                                  2, 512, rs)
    (tuv * torch.from_numpy(mesh.weights).cuda()).sum().backward()
    plain = rtx.trace(rs.scene, rays, "alpha", alpha_min=128)
    torch.cuda.synchronize()
    assert torch.equal(prim, plain[:, 1].view(torch.int32))
    assert torch.isfinite(moved.grad).all() and torch.isfinite(r2.grad).all()
    assert moved.grad.abs().sum() > 0
