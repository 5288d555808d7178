"""Pins of the instancing oracles: hand-derived translated and rotated
instances, an identity instance equal to the plain traversal of its mesh, and
the float32 two-level traversal (oracle B) against the float64 definition
(oracle A) on random instanced scenes."""
import numpy as np

from paper_1912_12786_amd import workloads as W
from tests.golden.load import load, uniform_alpha_textures

MISS = 0xFFFFFFFF


def world_boxes(mesh, maps):
    """World boxes of instances of `mesh` under object_from_world maps."""
    m = np.asarray(maps, np.float64).reshape(-1, 3, 4)
    wfo = np.concatenate([np.linalg.inv(m[:, :, :3]),
                          -np.einsum("nij,nj->ni", np.linalg.inv(m[:, :, :3]), m[:, :, 3])[..., None]], 2)
    lo = mesh.reshape(-1, 3).min(0).astype(np.float64)
    hi = mesh.reshape(-1, 3).max(0).astype(np.float64)
    n = m.shape[0]
    _, wlo, whi = W.instance_transforms(wfo, np.tile(lo, (n, 1)), np.tile(hi, (n, 1)))
    return wlo, whi


def test_golden_instances(oracle_lib):
    fx = load("instances.json")
    mesh = fx["vertices"]
    bvh = oracle_lib.build_bvh(mesh)
    for case in fx["cases"]:
        maps = np.asarray(case["maps"], np.float32)
        ids = np.zeros(len(maps), np.uint32)
        lo, hi = world_boxes(mesh, maps)
        tl = oracle_lib.build_tlas(lo, hi)
        B = oracle_lib.traverse_instanced([mesh], [bvh], ids, maps, tl, fx["rays"])
        A = oracle_lib.brute_instanced([mesh], ids, maps, fx["rays"])
        for R in (A, B):
            assert (int(R["inst"][0]), int(R["prim"][0])) == (case["inst"], case["prim"]), case
            assert (R["t"][0], R["u"][0], R["v"][0]) == (case["t"], case["u"], case["v"]), case


def test_identity_instance_equals_plain_traversal(oracle_lib):
    wl = W.tiny()
    mesh = wl.vertices
    bvh = oracle_lib.build_bvh(mesh)
    maps = np.array([[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]], np.float32)
    lo, hi = world_boxes(mesh, maps)
    tl = oracle_lib.build_tlas(lo, hi)
    B = oracle_lib.traverse_instanced([mesh], [bvh], np.zeros(1, np.uint32), maps, tl, wl.rays)
    P = oracle_lib.traverse(mesh, bvh, wl.rays)
    assert np.array_equal(B["prim"], P["prim"])
    for k in ("t", "u", "v"):
        assert np.array_equal(B[k].view(np.uint32), P[k].view(np.uint32))
    hit = P["prim"] != MISS
    assert np.all(B["inst"][hit] == 0) and np.all(B["inst"][~hit] == MISS)
    # the top-level root test comes first: a ray that misses it counts that one
    # test (as the plain traversal counts its missed root); otherwise one more
    # box test than the plain traversal
    assert np.array_equal(B["counters"][:, 1:], P["counters"][:, 1:])
    extra = B["counters"][:, 0].astype(np.int64) - P["counters"][:, 0]
    assert np.all((extra == 1) | ((extra == 0) & (P["counters"][:, 0] == 1)))
    assert (extra == 1).sum() > 0.5 * len(extra)


def test_instanced_oracle_b_matches_a(oracle_lib):
    for n_inst, kind in ((40, "default"), (60, "procedural")):
        wl = W.instanced(n_inst, 48, 27)
        bvhs = [oracle_lib.build_bvh(b) for b in wl["blas"]]
        tl = oracle_lib.build_tlas(wl["world_lo"], wl["world_hi"])
        # aim half the rays at instance centres so that many rays hit
        rng = np.random.default_rng(n_inst)
        rays = wl["rays"].copy()
        tgt = wl["world_from_object"][rng.integers(0, n_inst, size=rays.shape[0] // 2), :, 3]
        d = tgt - rays[: len(tgt), :3].astype(np.float64)
        rays[: len(tgt), 4:7] = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
        B = oracle_lib.traverse_instanced(wl["blas"], bvhs, wl["inst_blas"], wl["inst_m"], tl, rays,
                                          kind)
        A = oracle_lib.brute_instanced(wl["blas"], wl["inst_blas"], wl["inst_m"], rays, kind)
        ok = A["flags"] == 0
        assert ok.mean() > 0.9
        assert np.array_equal(A["prim"][ok], B["prim"][ok])
        assert np.array_equal(A["inst"][ok], B["inst"][ok])
        hit = ok & (A["prim"] != MISS)
        assert hit.sum() > 100
        assert np.all(np.abs(A["t"][hit] - B["t"][hit]) <= 1e-5 * A["t"][hit] + 1e-6)
        # any-hit answers the same occlusion question
        Ba = oracle_lib.traverse_instanced(wl["blas"], bvhs, wl["inst_blas"], wl["inst_m"], tl,
                                           rays, kind, any_hit=True)
        assert np.array_equal(Ba["prim"] == MISS, B["prim"] == MISS)


def _billboard_meshes():
    """The transparent-billboard fixture split into two meshes: the
    transparent quad Q0 (texture 0) and the opaque quad Q1 (texture 1)
    modelled at z = 0 and placed at z = -1 by its instance map."""
    fx = load("transparent_billboard.json")
    v = fx["vertices"]
    mesh_a = v[:2]
    mesh_b = v[2:].copy()
    mesh_b[:, :, 2] += 1.0                           # Q1 in its own object space
    tex = uniform_alpha_textures(fx["texture_alpha"], fx["texture_size"])
    tc = fx["texcoords"]
    ident = [1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]
    up = [1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 1]        # world z = -1 -> object z = 0
    maps = np.array([ident, up], np.float32)
    return fx, [mesh_a, mesh_b], [fx["geom_ids"][:2], fx["geom_ids"][2:]], [tc[:2], tc[2:]], tex, maps


def test_alpha_instances_golden(oracle_lib):
    """Section 4's alpha mask per instanced mesh (Section 3.2): the same hits
    as the single-scene fixture, now found in the second instance, with
    counts derived by hand: TLAS root (a leaf of both instances), then each
    instance's root box and leaf."""
    fx, meshes, geoms, tcs, tex, maps = _billboard_meshes()
    ids = np.array([0, 1], np.uint32)
    lo = np.array([[-1, -1, 0], [-1, -1, -1]], np.float32) - 1e-3
    hi = np.array([[1, 1, 0], [1, 1, -1]], np.float32) + 1e-3
    tl = oracle_lib.build_tlas(lo, hi)
    bvhs = [oracle_lib.build_bvh(m) for m in meshes]
    akw = dict(geom_ids=geoms, texcoords=tcs, textures=tex, alpha_min=128)
    Ba = oracle_lib.traverse_instanced(meshes, bvhs, ids, maps, tl, fx["rays"], "alpha", **akw)
    Aa = oracle_lib.brute_instanced(meshes, ids, maps, fx["rays"], "alpha", **akw)
    for R in (Aa, Ba):
        assert (int(R["inst"][0]), int(R["prim"][0])) == (1, 1)
        assert (R["t"][0], R["u"][0], R["v"][0]) == (2.0, 0.625, 0.0625)
    # TLAS root; instance 0: root + 2 triangles, the candidate rejected;
    # instance 1: root + 2 triangles, the candidate accepted
    assert Ba["counters"][0].tolist() == [3, 4, 2, 1]
    Bd = oracle_lib.traverse_instanced(meshes, bvhs, ids, maps, tl, fx["rays"], "default")
    assert (int(Bd["inst"][0]), int(Bd["prim"][0]), Bd["t"][0]) == (0, 1, 1.0)
    # instance 1's root box lies beyond the accepted t = 1: missed, no triangles
    assert Bd["counters"][0].tolist() == [3, 2, 1, 1]


def test_alpha_identity_instance_equals_plain(oracle_lib):
    wl = W.tiny()
    rng = np.random.default_rng(4)
    tex = W.alpha_textures(4, 64, 4)
    geom = rng.integers(0, 4, size=wl.n_tris).astype(np.uint32)
    tc = rng.uniform(0, 1, size=(wl.n_tris, 3, 2)).astype(np.float32)
    bvh = oracle_lib.build_bvh(wl.vertices)
    maps = np.array([[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]], np.float32)
    lo, hi = world_boxes(wl.vertices, maps)
    tl = oracle_lib.build_tlas(lo, hi)
    B = oracle_lib.traverse_instanced([wl.vertices], [bvh], np.zeros(1, np.uint32), maps, tl,
                                      wl.rays, "alpha", geom_ids=[geom], texcoords=[tc],
                                      textures=tex, alpha_min=128)
    Pl = oracle_lib.traverse(wl.vertices, bvh, wl.rays, "alpha", geom_ids=geom, texcoords=tc,
                             textures=tex, alpha_min=128)
    assert np.array_equal(B["prim"], Pl["prim"])
    for k in ("t", "u", "v"):
        assert np.array_equal(B[k].view(np.uint32), Pl[k].view(np.uint32))
    assert np.array_equal(B["counters"][:, 1:], Pl["counters"][:, 1:])
    assert (Pl["counters"][:, 3] > 0).sum() > 50        # the mask accepts and rejects
    assert (Pl["counters"][:, 2] > Pl["counters"][:, 3]).sum() > 50


def test_alpha_instanced_b_matches_a(oracle_lib):
    wl = W.instanced(40, 48, 27)
    rng = np.random.default_rng(40)
    tex = W.alpha_textures(3, 64, 40)
    geoms = [rng.integers(0, 3, size=m.shape[0]).astype(np.uint32) for m in wl["blas"]]
    tcs = [rng.uniform(0, 1, size=(m.shape[0], 3, 2)).astype(np.float32) for m in wl["blas"]]
    bvhs = [oracle_lib.build_bvh(b) for b in wl["blas"]]
    tl = oracle_lib.build_tlas(wl["world_lo"], wl["world_hi"])
    rays = wl["rays"].copy()
    tgt = wl["world_from_object"][rng.integers(0, 40, size=rays.shape[0] // 2), :, 3]
    d = tgt - rays[: len(tgt), :3].astype(np.float64)
    rays[: len(tgt), 4:7] = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    kw = dict(geom_ids=geoms, texcoords=tcs, textures=tex, alpha_min=128)
    B = oracle_lib.traverse_instanced(wl["blas"], bvhs, wl["inst_blas"], wl["inst_m"], tl, rays,
                                      "alpha", **kw)
    A = oracle_lib.brute_instanced(wl["blas"], wl["inst_blas"], wl["inst_m"], rays, "alpha", **kw)
    ok = A["flags"] == 0
    assert ok.mean() > 0.85
    assert np.array_equal(A["prim"][ok], B["prim"][ok])
    assert np.array_equal(A["inst"][ok], B["inst"][ok])
    hit = ok & (A["prim"] != MISS)
    assert hit.sum() > 100
    assert np.all(np.abs(A["t"][hit] - B["t"][hit]) <= 1e-5 * A["t"][hit] + 1e-6)
    # the mask matters: some rays pass a rejected candidate
    assert (B["counters"][:, 2] > B["counters"][:, 3]).sum() > 50
