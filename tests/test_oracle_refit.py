"""Pins of oracle B's refit (new vertex positions, same tree; not in the
paper, whose BVH construction is open).

Refitting to the build's own vertices reproduces the builder's boxes bit for
bit (the builder grows every node box over its triangles with the same
strict comparisons); after random moves every box equals the exact min/max
over its subtree's vertices (numpy reductions on the leaf ranges) with the
first-occurrence sign of zero, invalid indices add nothing, and traversing the
refitted tree gives oracle A's closest hits on the moved mesh."""
import numpy as np
import pytest

from tests.test_oracle_pins import _random_scene

MISS = 0xFFFFFFFF


def _indexed(soup):
    """An indexed mesh with one vertex per corner of a triangle soup."""
    v = np.ascontiguousarray(soup, np.float32).reshape(-1, 3)
    return v, np.arange(v.shape[0], dtype=np.uint32).reshape(-1, 3)


def _subtree_ranges(nodes):
    """[first, end) of each node's triangles in leaf order (preorder ids)."""
    first = np.zeros(len(nodes), np.int64)
    end = np.zeros(len(nodes), np.int64)
    for k in range(len(nodes) - 1, -1, -1):
        if nodes[k]["count"]:
            first[k], end[k] = nodes[k]["first"], nodes[k]["first"] + nodes[k]["count"]
        else:
            first[k] = first[nodes[k]["left"]]
            end[k] = end[nodes[k]["right"]]
    return first, end


@pytest.mark.parametrize("seed,n,max_leaf", [(1, 300, 4), (2, 1000, 2), (3, 17, 1), (4, 5, 7)])
def test_refit_identity_reproduces_build(oracle_lib, seed, n, max_leaf):
    rng = np.random.default_rng(seed)
    verts, _ = _random_scene(rng, n, 1)
    bvh = oracle_lib.build_bvh(verts, max_leaf=max_leaf)
    v, f = _indexed(verts)
    R = oracle_lib.refit(bvh, v, f)
    for key in ("lo", "hi"):
        assert np.array_equal(R.nodes[key].view(np.uint32), bvh.nodes[key].view(np.uint32))
    for key in ("left", "right", "first", "count", "depth"):
        assert np.array_equal(R.nodes[key], bvh.nodes[key])


@pytest.mark.parametrize("seed", range(4))
def test_refit_boxes_are_subtree_extents(oracle_lib, seed):
    rng = np.random.default_rng(10 + seed)
    verts, _ = _random_scene(rng, 800, 1)
    bvh = oracle_lib.build_bvh(verts, max_leaf=2)
    v, f = _indexed(verts)
    moved = (v + rng.normal(0.0, 0.05, size=v.shape)).astype(np.float32)
    R = oracle_lib.refit(bvh, moved, f)
    first, end = _subtree_ranges(bvh.nodes)
    corners = moved[f[bvh.perm]]                      # leaf order, [n, 3, 3]
    for k in range(bvh.n_nodes):
        pts = corners[first[k]:end[k]].reshape(-1, 3)
        assert np.array_equal(R.nodes["lo"][k], pts.min(0))
        assert np.array_equal(R.nodes["hi"][k], pts.max(0))


def test_refit_zero_sign_and_invalid_indices(oracle_lib):
    """Two triangles in one leaf, the first touching x = +0, the second
    x = -0: the lower bound keeps +0 (the first occurrence); swapped, -0.  A
    corner with an index past the vertices adds nothing to the box."""
    v = np.array([[+0.0, 0, 0], [1, 0, 0], [1, 1, 0],
                  [-0.0, 0, 1], [1, 0, 1], [1, 1, 1]], np.float32)
    for order, sign in (([0, 1], 0), ([1, 0], 1)):
        f = np.array([[0, 1, 2], [3, 4, 5]], np.uint32)[order]
        soup = v[f]
        bvh = oracle_lib.build_bvh(soup, max_leaf=2)
        assert bvh.nodes[0]["count"] == 2
        R = oracle_lib.refit(bvh, v, f)
        lo_x = R.nodes["lo"][0][0]
        assert lo_x == 0.0 and np.signbit(lo_x) == bool(sign)
    # vertices 0 and 7 lie outside every triangle: reading either for the
    # invalid index (a zero default, a clamp to the last vertex) would show
    w = np.concatenate([[[-5.0, -5.0, -5.0]], v, [[7.0, 7.0, 7.0]]]).astype(np.float32)
    f = np.array([[1, 2, 3], [4, 5, 99]], np.uint32)
    bvh = oracle_lib.build_bvh(w[np.array([[1, 2, 3], [4, 5, 6]])], max_leaf=2)
    R = oracle_lib.refit(bvh, w, f)
    assert np.array_equal(R.nodes["lo"][0], [0, 0, 0]) and np.array_equal(R.nodes["hi"][0], [1, 1, 1])


@pytest.mark.parametrize("kind", ["default", "alpha", "procedural"])
def test_refit_traversal_matches_oracle_a(oracle_lib, kind):
    """The tree built on one mesh and refitted to a moved copy finds oracle
    A's closest hits on the moved mesh (the boxes stay exact, only their
    quality drops)."""
    from tests.test_oracle_pins import _scene_params
    for seed in range(4):
        rng = np.random.default_rng(40 + seed)
        verts, rays = _random_scene(rng, int(rng.integers(20, 200)), 400)
        kw = _scene_params(rng, kind, verts.shape[0])
        bvh = oracle_lib.build_bvh(verts, max_leaf=2)
        v, f = _indexed(verts)
        moved = (v + rng.normal(0.0, 0.1, size=v.shape)).astype(np.float32)
        R = oracle_lib.refit(bvh, moved, f)
        soup = moved[f]
        A = oracle_lib.brute(soup, rays, kind, **kw)
        B = oracle_lib.traverse(soup, R, rays, kind, **kw)
        ok = A["flags"] == 0
        assert np.array_equal(A["prim"][ok], B["prim"][ok])
        hit = ok & (A["prim"] != MISS)
        tol_t = np.maximum(1e-5 * np.abs(A["t"][hit]), A["bound_t"][hit])
        assert np.all(np.abs(B["t"][hit] - A["t"][hit]) <= tol_t)
        # the same tree without the refit misses some of them
        stale = oracle_lib.traverse(soup, bvh, rays, kind, **kw)
        assert not np.array_equal(stale["prim"], B["prim"])
