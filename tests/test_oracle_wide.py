"""Pins of oracle B's four-wide layout (the BVH's arity is left open by
Section 3.2; the layout collapses the binary BVH into nodes of up to four
children).

* hand-derived scenes (tests/golden/wide_nodes.json): the collapse (largest
  surface area first, ties to the earlier entry; fewer than four children
  when no inner entry is left), the stack bound, and the hits and exact
  counters of rays whose counts tell the wide traversal's order (all
  children tested, nearest first, second nearest on top) from the binary
  one's;
* properties of the collapse on random scenes that follow from its
  definition without re-running it: every binary leaf reached exactly once,
  child lists in the binary left-to-right order, fewer than four children
  only when all are leaves, every expanded node at least as large as every
  inner child left, and the stack bound equal to the largest sum of k - 1
  along a root-to-leaf path;
* counts of traversals without accepts against the order-free set formula;
* hits against the float64 definition (oracle A) outside the exception set,
  and against the binary traversal, for every intersector and query.
"""
import numpy as np
import pytest

from tests.golden.load import load, uniform_alpha_textures

MISS = 0xFFFFFFFF


def _leaf_tris(bvh, node):
    nd = bvh.nodes[node]
    assert nd["count"] > 0
    return sorted(int(bvh.perm[j]) for j in range(nd["first"], nd["first"] + nd["count"]))


@pytest.mark.parametrize("scene", ["four", "three", "tie", "dup"])
def test_golden_wide_nodes(oracle_lib, scene):
    fx = load("wide_nodes.json")
    sc = fx["scenes"][scene]
    verts = np.asarray(sc["vertices"], np.float32)
    rays = np.asarray([[np.inf if x == "inf" else x for x in r] for r in sc["rays"]], np.float32)
    bvh = oracle_lib.build_bvh(verts, max_leaf=2)
    w = oracle_lib.widen(bvh)
    assert w["order"][0] == 0
    root = w["wide"][0]
    assert root["n"] == sc["wide_children"]
    kids = [int(c) for c in root["child"][: root["n"]]]
    got = [_leaf_tris(bvh, c) if bvh.nodes[c]["count"] else "inner" for c in kids]
    assert got == sc["leaves"]
    assert len(w["order"]) == 1 + sc["leaves"].count("inner")
    assert w["stack_bound"] == sc["stack_bound"]
    for layout, key in (("wide4", "wide"), ("f32", "binary")):
        B = oracle_lib.traverse(verts, bvh, rays, layout=layout)
        for case in sc["cases"]:
            i = case["ray"]
            assert B["counters"][i].tolist() == case[key], (layout, i, B["counters"][i])
            if case.get("miss"):
                assert B["prim"][i] == MISS
            else:
                assert B["prim"][i] == case["prim"]
                for k in ("t", "u", "v"):
                    assert float(B[k][i]) == case[k], (layout, i, k)
    # any hit: the first accepted hit in the wide order is the same triangle
    Ba = oracle_lib.traverse(verts, bvh, rays, layout="wide4", any_hit=True)
    for case in sc["cases"]:
        assert Ba["prim"][case["ray"]] == (MISS if case.get("miss") else case["prim"])


def _area(lo, hi):
    d = hi.astype(np.float64) - lo.astype(np.float64)
    return 2.0 * (d[0] * d[1] + d[1] * d[2] + d[2] * d[0])


def _frontier_paths(nodes, head, kids):
    """Binary inner nodes strictly between head and its wide children, and
    the children in the binary left-to-right order of the collapsed
    subtree."""
    kidset = set(kids)
    absorbed, order = [], []

    def rec(x):
        if x in kidset:
            order.append(x)
            return
        assert nodes["count"][x] == 0, "a wide child list skipped a leaf"
        absorbed.append(x)
        rec(int(nodes["left"][x]))
        rec(int(nodes["right"][x]))

    rec(int(nodes["left"][head]))
    rec(int(nodes["right"][head]))
    return absorbed, order


def _check_wide(bvh, w):
    nodes = bvh.nodes
    wide = w["wide"]
    heads = set(int(h) for h in w["order"])
    if bvh.n_nodes <= 1 or nodes["count"][0] > 0:
        assert len(heads) == 0 and w["stack_bound"] == 0
        return
    assert w["order"][0] == 0
    leaves_seen = []
    preorder = []

    def walk(h, pushed):
        preorder.append(h)
        k = int(wide[h]["n"])
        assert 2 <= k <= 4
        kids = [int(c) for c in wide[h]["child"][:k]]
        absorbed, order = _frontier_paths(nodes, h, kids)
        assert order == kids, "children not in the binary left-to-right order"
        assert len(absorbed) == k - 2
        inner_kids = [c for c in kids if nodes["count"][c] == 0]
        if k < 4:
            assert not inner_kids, "fewer than four children while an inner entry remains"
        if absorbed and inner_kids:
            a_min = min(_area(nodes["lo"][x], nodes["hi"][x]) for x in absorbed)
            r_max = max(_area(nodes["lo"][x], nodes["hi"][x]) for x in inner_kids)
            assert a_min >= r_max, "a larger inner entry was left unexpanded"
        best = 0
        for c in kids:
            if nodes["count"][c] > 0:
                leaves_seen.append(c)
                best = max(best, pushed + k - 1)
            else:
                assert c in heads
                best = max(best, walk(c, pushed + k - 1))
        return best

    bound = walk(0, 0)
    assert preorder == [int(h) for h in w["order"]], "wide nodes not in depth-first preorder"
    assert bound == w["stack_bound"]
    all_leaves = [i for i in range(bvh.n_nodes) if nodes["count"][i] > 0]
    assert sorted(leaves_seen) == all_leaves


@pytest.mark.parametrize("seed,n,max_leaf", [(1, 7, 1), (2, 100, 2), (3, 1000, 4), (4, 5000, 1),
                                             (5, 3, 4), (6, 9, 2)])
def test_widen_properties_random(oracle_lib, seed, n, max_leaf):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0, 10, size=(n, 1, 3))
    v = (c + rng.normal(scale=rng.uniform(0.01, 1.0, size=(n, 1, 1)), size=(n, 3, 3))).astype(np.float32)
    bvh = oracle_lib.build_bvh(v, max_leaf=max_leaf)
    _check_wide(bvh, oracle_lib.widen(bvh))


def test_widen_workloads(oracle_lib):
    from paper_1912_12786_amd import workloads as W
    wl = W.tiny()
    for ml in (1, 2, 4):
        bvh = oracle_lib.build_bvh(wl.vertices, max_leaf=ml)
        _check_wide(bvh, oracle_lib.widen(bvh))
    bb = W.billboards(n_quads=2000, width=32, height=18)
    bvh = oracle_lib.build_bvh(bb.vertices, max_leaf=2)
    _check_wide(bvh, oracle_lib.widen(bvh))


def test_widen_root_leaf_and_empty(oracle_lib):
    v = np.zeros((3, 3, 3), np.float32)
    v[:, 1, 0] = 1
    v[:, 2, 1] = 1
    bvh = oracle_lib.build_bvh(v)
    w = oracle_lib.widen(bvh)
    assert len(w["order"]) == 0 and w["stack_bound"] == 0
    r = np.array([[0.2, 0.2, 1, 0, 0, 0, -1, np.inf]], np.float32)
    B = oracle_lib.traverse(v, bvh, r, layout="wide4")
    assert B["counters"][0].tolist() == [1, 3, 1, 1]
    e = oracle_lib.build_bvh(np.zeros((0, 3, 3), np.float32))
    assert len(oracle_lib.widen(e)["order"]) == 0


def _slab64(lo, hi, o, d):
    tiny = 2.0 ** -80
    dd = np.where(np.abs(d) < tiny, np.copysign(tiny, d), d)
    t0 = (lo - o) / dd
    t1 = (hi - o) / dd
    return max(np.max(np.minimum(t0, t1)), 0.0), np.min(np.maximum(t0, t1))


def test_wide_counts_without_accepts_follow_set_formula(oracle_lib):
    """Every candidate rejected: tmax never shrinks, so a wide node is
    entered iff its box (as a child) and its ancestors' are hit; then
    boxes = 1 + sum of k over the entered wide nodes and triangles = the
    entered leaves' sizes."""
    from paper_1912_12786_amd import workloads as W
    wl = W.tiny()
    verts = wl.vertices
    n = verts.shape[0]
    kw = dict(geom_ids=np.zeros(n, np.uint32), texcoords=np.zeros((n, 3, 2), np.float32),
              textures=uniform_alpha_textures([0], (2, 2)), alpha_min=1)
    bvh = oracle_lib.build_bvh(verts, max_leaf=2)
    w = oracle_lib.widen(bvh)
    rays = wl.rays[::5]
    B = oracle_lib.traverse(verts, bvh, rays, "alpha", layout="wide4", **kw)
    assert np.all(B["prim"] == MISS)
    nodes = bvh.nodes
    lo, hi = nodes["lo"].astype(np.float64), nodes["hi"].astype(np.float64)
    checked = 0
    for i in range(rays.shape[0]):
        o, d = rays[i, :3].astype(np.float64), rays[i, 4:7].astype(np.float64)
        grazing = False

        def hit(x):
            nonlocal grazing
            tn, tf = _slab64(lo[x], hi[x], o, d)
            if abs(tn - tf) <= 1e-5 * max(1.0, abs(tn)):
                grazing = True
            return tn <= tf

        boxes, tris = 1, 0
        todo = [0] if hit(0) else []
        while todo:
            x = todo.pop()
            if nodes["count"][x] > 0:
                tris += int(nodes["count"][x])
                continue
            k = int(w["wide"][x]["n"])
            boxes += k
            todo += [int(c) for c in w["wide"][x]["child"][:k] if hit(int(c))]
        if grazing:
            continue
        checked += 1
        assert B["counters"][i, 0] == boxes, i
        assert B["counters"][i, 1] == tris, i
    assert checked > 0.9 * rays.shape[0]


def _scene(rng, kind, n_tris, n_rays):
    c = rng.uniform(0, 1, size=(n_tris, 1, 3))
    v = (c + rng.normal(scale=0.15, size=(n_tris, 3, 3))).astype(np.float32)
    o = rng.uniform(-0.5, 1.5, size=(n_rays, 3))
    d = rng.normal(size=(n_rays, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = np.zeros((n_rays, 8), np.float32)
    r[:, 0:3], r[:, 4:7], r[:, 7] = o, d, np.inf
    kw = {}
    if kind == "alpha":
        tex = rng.integers(0, 256, size=(3, 8, 8)).astype(np.uint32) << np.uint32(24)
        kw = dict(geom_ids=rng.integers(0, 3, size=n_tris).astype(np.uint32),
                  texcoords=rng.uniform(0, 1, size=(n_tris, 3, 2)).astype(np.float32),
                  textures=tex, alpha_min=128)
    return v, r, kw


@pytest.mark.parametrize("kind", ["default", "alpha", "procedural"])
@pytest.mark.parametrize("seed", [11, 12])
def test_wide_matches_definition_and_binary(oracle_lib, kind, seed):
    rng = np.random.default_rng(seed)
    v, r, kw = _scene(rng, kind, 300, 2000)
    bvh = oracle_lib.build_bvh(v, max_leaf=1 + seed % 3)
    A = oracle_lib.brute(v, r, kind, **kw)
    Bw = oracle_lib.traverse(v, bvh, r, kind, layout="wide4", **kw)
    Bb = oracle_lib.traverse(v, bvh, r, kind, **kw)
    ok = A["flags"] == 0
    assert np.array_equal(Bw["prim"][ok], A["prim"][ok])
    # the binary traversal reaches the same nearest accepted hit; only an
    # exact tie in t could pick another triangle
    same = Bw["prim"] == Bb["prim"]
    assert np.all(same | (Bw["t"] == Bb["t"]))
    assert np.array_equal(Bw["t"].view(np.uint32), Bb["t"].view(np.uint32))
    Aw = oracle_lib.traverse(v, bvh, r, kind, layout="wide4", any_hit=True, **kw)
    assert np.array_equal(Aw["prim"] != MISS, Bw["prim"] != MISS)
    Mw = oracle_lib.traverse(v, bvh, r, kind, layout="wide4", multi_k=3, **kw)
    Mb = oracle_lib.traverse(v, bvh, r, kind, multi_k=3, **kw)
    assert np.array_equal(Mw["n_hits"], Mb["n_hits"])
    assert np.array_equal(Mw["t"].view(np.uint32), Mb["t"].view(np.uint32))
    # the wide traversal fetches fewer nodes
    nb = (Bb["counters"][:, 0].astype(np.int64) - 1) // 2
    assert Bw["counters"][:, 0].sum() <= 1.5 * Bb["counters"][:, 0].sum()
    assert nb.sum() > 0
