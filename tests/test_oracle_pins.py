"""Pins of the CPU oracle to facts that do not come from the oracle itself.

* hand-derived closed-form cases (tests/golden/*.json, each citing the paper);
* oracle A's float64 plane test against LAPACK (numpy.linalg.solve) of the
  3x3 system o + t d = v0 + u e1 + v e2;
* oracle A's nearest accepted hit against an independent numpy brute force;
* oracle B (float32 BVH traversal) against oracle A outside the exception set;
* any-hit <=> closest-hit;
* the counts of a traversal in which no candidate is ever accepted, against
  the order-free set formula (a node is entered iff its box and all its
  ancestors' boxes are hit);
* the exception flags on constructed ties and edge hits.
"""
import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from tests.golden.load import load, uniform_alpha_textures

MISS = 0xFFFFFFFF


# ----------------------------------------------------------------------------
# golden closed-form cases
# ----------------------------------------------------------------------------
def _check_accept(res, i, accept, exact, rtol=0.0, atol=0.0):
    prim = int(res["prim"][i])
    cands = {a["prim"]: a for a in accept}
    assert prim in cands, f"prim {prim} not in {sorted(cands)}"
    a = cands[prim]
    for k in ("t", "u", "v"):
        got = float(res[k][i])
        if exact:
            assert got == a[k], (k, got, a[k])
        else:
            assert abs(got - a[k]) <= atol + rtol * abs(a[k]), (k, got, a[k])


def test_golden_quad_centre(oracle_lib):
    fx = load("quad_centre.json")
    bvh = oracle_lib.build_bvh(fx["vertices"])
    A = oracle_lib.brute(fx["vertices"], fx["rays"])
    B = oracle_lib.traverse(fx["vertices"], bvh, fx["rays"])
    for case in fx["cases"]:
        i = case["ray"]
        if case.get("miss"):
            assert A["prim"][i] == MISS and B["prim"][i] == MISS, i
            continue
        _check_accept(A, i, case["accept"], case["exact"])
        _check_accept(B, i, case["accept"], case["exact"])
        if "oracle_b_prim" in case:
            assert B["prim"][i] == case["oracle_b_prim"]
        if case.get("flags_none"):
            assert A["flags"][i] == 0
        if "flags_any" in case:
            assert A["flags"][i] != 0
    # the tie on the diagonal is flagged as a near-tie (both prims at t=1)
    assert A["flags"][0] & oracle_lib.E_NEAR_TIE


def test_golden_shared_edge(oracle_lib):
    fx = load("shared_edge.json")
    bvh = oracle_lib.build_bvh(fx["vertices"])
    A = oracle_lib.brute(fx["vertices"], fx["rays"])
    B = oracle_lib.traverse(fx["vertices"], bvh, fx["rays"])
    c0, c1 = fx["cases"]
    _check_accept(A, 0, c0["accept"], True)
    _check_accept(B, 0, c0["accept"], True)
    assert A["flags"][0] & oracle_lib.E_NEAR_EDGE
    for R in (A, B):
        assert R["prim"][1] == MISS and math.isinf(R["t"][1])


def test_golden_transparent_billboard(oracle_lib):
    fx = load("transparent_billboard.json")
    tex = uniform_alpha_textures(fx["texture_alpha"], fx["texture_size"])
    for case in fx["cases"]:
        sel = case.get("only_prims", list(range(len(fx["vertices"]))))
        verts = fx["vertices"][sel]
        kw = {}
        if case["intersector"] == "alpha":
            kw = dict(geom_ids=fx["geom_ids"][sel], texcoords=fx["texcoords"][sel], textures=tex,
                      alpha_min=case["alpha_min"])
        bvh = oracle_lib.build_bvh(verts)
        A = oracle_lib.brute(verts, fx["rays"], case["intersector"], **kw)
        B = oracle_lib.traverse(verts, bvh, fx["rays"], case["intersector"], **kw)
        if case.get("miss"):
            assert A["prim"][0] == MISS and B["prim"][0] == MISS
        else:
            _check_accept(A, 0, case["accept"], True)
            _check_accept(B, 0, case["accept"], True)
        assert B["counters"][0].tolist() == case["counters"]


def test_golden_alpha_threshold(oracle_lib):
    fx = load("alpha_threshold.json")
    for case in fx["cases"]:
        tex = uniform_alpha_textures([case["a8"]], fx["texture_size"])
        kw = dict(geom_ids=fx["geom_ids"], texcoords=fx["texcoords"], textures=tex,
                  alpha_min=case["alpha_min"])
        bvh = oracle_lib.build_bvh(fx["vertices"])
        A = oracle_lib.brute(fx["vertices"], fx["rays"], "alpha", **kw)
        B = oracle_lib.traverse(fx["vertices"], bvh, fx["rays"], "alpha", **kw)
        for R in (A, B):
            assert (R["prim"][0] != MISS) == case["hit"], case


def test_alpha_threshold_byte_mapping():
    # a float threshold tau on a8/255 is the integer test a8 >= ceil(255 tau)
    for tau, expect in ((0.5, 128), (0.01, 3)):
        m = math.ceil(255 * tau)
        assert m == expect
        assert (m - 1) / 255 < tau <= m / 255


def test_golden_procedural_checker(oracle_lib):
    fx = load("procedural_checker.json")
    rays = np.array([[x, y, 1, 0, 0, 0, -1, np.inf] for x, y, _ in fx["points"]], np.float32)
    bvh = oracle_lib.build_bvh(fx["vertices"])
    A = oracle_lib.brute(fx["vertices"], rays, "procedural", checker_n=fx["checker_n"])
    B = oracle_lib.traverse(fx["vertices"], bvh, rays, "procedural", checker_n=fx["checker_n"])
    for i, (x, y, vis) in enumerate(fx["points"]):
        for R in (A, B):
            assert (R["prim"][i] != MISS) == vis, (x, y)
            if vis:
                assert abs(R["u"][i] - x) < 1e-6 and abs(R["v"][i] - y) < 1e-6


def test_golden_two_leaf_counts(oracle_lib):
    fx = load("two_leaf_counts.json")
    bvh = oracle_lib.build_bvh(fx["vertices"])
    exp = fx["bvh"]
    assert bvh.n_nodes == exp["n_nodes"]
    root, left, right = bvh.nodes[0], bvh.nodes[bvh.nodes[0]["left"]], bvh.nodes[bvh.nodes[0]["right"]]
    assert root["count"] == 0
    assert sorted(bvh.perm[left["first"]:left["first"] + left["count"]].tolist()) == exp["left_prims"]
    assert sorted(bvh.perm[right["first"]:right["first"] + right["count"]].tolist()) == exp["right_prims"]
    B = oracle_lib.traverse(fx["vertices"], bvh, fx["rays"])
    A = oracle_lib.brute(fx["vertices"], fx["rays"])
    for case in fx["cases"]:
        i = case["ray"]
        assert B["counters"][i].tolist() == case["counters"], case
        for R in (A, B):
            if case.get("miss"):
                assert R["prim"][i] == MISS
            else:
                assert R["prim"][i] == case["prim"]
                rt, at = case.get("t_rtol", 0.0), case.get("uv_atol", 0.0)
                assert abs(R["t"][i] - case["t"]) <= rt * case["t"]
                assert abs(R["u"][i] - case["u"]) <= at and abs(R["v"][i] - case["v"]) <= at


def test_empty_scene(oracle_lib):
    verts = np.zeros((0, 3, 3), np.float32)
    rays = np.array([[0, 0, 1, 0, 0, 0, -1, np.inf]], np.float32)
    bvh = oracle_lib.build_bvh(verts)
    B = oracle_lib.traverse(verts, bvh, rays)
    A = oracle_lib.brute(verts, rays)
    assert B["prim"][0] == MISS and A["prim"][0] == MISS
    assert B["counters"][0].tolist() == [0, 0, 0, 0]


# ----------------------------------------------------------------------------
# oracle A against LAPACK
# ----------------------------------------------------------------------------
def _solve_tuv(o, d, tri):
    """o + t d = v0 + u e1 + v e2  <=>  [d, -e1, -e2] (t,u,v) = v0 - o."""
    v0, v1, v2 = (tri[k].astype(np.float64) for k in range(3))
    M = np.stack([d, -(v1 - v0), -(v2 - v0)], axis=1)
    return np.linalg.solve(M, v0 - o)


def test_oracle_a_plane_test_matches_linalg(oracle_lib):
    rng = np.random.default_rng(11)
    tris = rng.uniform(-1, 1, size=(40, 3, 3)).astype(np.float32)
    checked = 0
    for k in range(tris.shape[0]):
        tri = tris[k:k + 1]
        cen = tri[0].astype(np.float64).mean(0)
        for _ in range(8):
            o = rng.uniform(-3, 3, size=3)
            # aim near the centroid so that many rays hit
            tgt = cen + rng.normal(0, 0.3, size=3)
            d = tgt - o
            d /= np.linalg.norm(d)
            ray = np.array([[*o, 0, *d, np.inf]], np.float32)
            o32 = ray[0, :3].astype(np.float64)
            d32 = ray[0, 4:7].astype(np.float64)
            t, u, v = _solve_tuv(o32, d32, tri[0])
            A = oracle_lib.brute(tri, ray)
            inside = u >= 0 and v >= 0 and u + v <= 1 and t > 0
            margin = min(u, v, 1 - u - v)
            if abs(margin) < 1e-9:
                continue
            assert (A["prim"][0] == 0) == inside
            if inside:
                checked += 1
                assert abs(A["t"][0] - t) <= 1e-9 * max(1, abs(t))
                assert abs(A["u"][0] - u) <= 1e-9 and abs(A["v"][0] - v) <= 1e-9
    assert checked > 50


def _random_scene(rng, n_tris, n_rays, size=(0.05, 0.6)):
    c = rng.uniform(0, 1, size=(n_tris, 1, 3))
    s = rng.uniform(size[0], size[1], size=(n_tris, 1, 1))
    verts = (c + s * rng.normal(0, 1, size=(n_tris, 3, 3))).astype(np.float32)
    o = rng.uniform(-1, 2, size=(n_rays, 3))
    tgt = rng.uniform(0, 1, size=(n_rays, 3))
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.zeros((n_rays, 8), np.float32)
    rays[:, :3] = o
    rays[:, 4:7] = d
    rays[:, 3] = 0.0
    rays[:, 7] = np.inf
    return verts, rays


def test_oracle_a_nearest_matches_numpy_bruteforce(oracle_lib):
    rng = np.random.default_rng(5)
    verts, rays = _random_scene(rng, 30, 200)
    A = oracle_lib.brute(verts, rays)
    agree = 0
    for i in range(rays.shape[0]):
        o = rays[i, :3].astype(np.float64)
        d = rays[i, 4:7].astype(np.float64)
        best_t, best_k, ambiguous = np.inf, MISS, False
        for k in range(verts.shape[0]):
            try:
                t, u, v = _solve_tuv(o, d, verts[k])
            except np.linalg.LinAlgError:
                continue
            m = min(u, v, 1 - u - v)
            if abs(m) < 1e-7:
                ambiguous = True
            if m >= 0 and t > 0:
                if abs(t - best_t) < 1e-7 * max(1, abs(t)):
                    ambiguous = True
                if t < best_t:
                    best_t, best_k = t, k
        if ambiguous:
            continue
        agree += 1
        assert A["prim"][i] == best_k, i
        if best_k != MISS:
            assert abs(A["t"][i] - best_t) <= 1e-9 * max(1.0, best_t)
    assert agree > 150


# ----------------------------------------------------------------------------
# oracle B against oracle A (brute force on small inputs)
# ----------------------------------------------------------------------------
def _scene_params(rng, kind, n_tris):
    kw = {}
    if kind == "alpha":
        n_tex = 3
        tex = np.zeros((n_tex, 8, 8), np.uint32)
        a8 = rng.integers(0, 256, size=(n_tex, 8, 8)).astype(np.uint32)
        tex[:] = (a8 << 24) | 0x00112233
        kw = dict(geom_ids=rng.integers(0, n_tex, size=n_tris).astype(np.uint32),
                  texcoords=rng.uniform(0, 1, size=(n_tris, 3, 2)).astype(np.float32),
                  textures=tex, alpha_min=int(rng.integers(1, 256)))
    elif kind == "procedural":
        kw = dict(checker_n=int(rng.integers(1, 12)))
    return kw


def _compare_a_b(oracle_lib, verts, rays, kind, kw, any_hit=False):
    bvh = oracle_lib.build_bvh(verts)
    A = oracle_lib.brute(verts, rays, kind, any_hit=any_hit, **kw)
    B = oracle_lib.traverse(verts, bvh, rays, kind, any_hit=any_hit, **kw)
    ok = A["flags"] == 0
    if any_hit:
        # the boolean answer is unique; B's occluder must be an accepted hit
        assert np.array_equal((A["prim"] == MISS)[ok], (B["prim"] == MISS)[ok])
        return ok.sum()
    assert np.array_equal(A["prim"][ok], B["prim"][ok])
    hit = ok & (A["prim"] != MISS)
    tol_t = np.maximum(1e-5 * np.abs(A["t"][hit]), A["bound_t"][hit])
    tol_uv = np.maximum(1e-5, A["bound_uv"][hit])
    assert np.all(np.abs(B["t"][hit] - A["t"][hit]) <= tol_t)
    assert np.all(np.abs(B["u"][hit] - A["u"][hit]) <= tol_uv)
    assert np.all(np.abs(B["v"][hit] - A["v"][hit]) <= tol_uv)
    return ok.sum()


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), n_tris=st.integers(1, 64),
       kind=st.sampled_from(["default", "alpha", "procedural"]),
       any_hit=st.booleans())
def test_oracle_b_matches_oracle_a(oracle_lib, seed, n_tris, kind, any_hit):
    rng = np.random.default_rng(seed)
    verts, rays = _random_scene(rng, n_tris, 256)
    kw = _scene_params(rng, kind, n_tris)
    _compare_a_b(oracle_lib, verts, rays, kind, kw, any_hit)


def test_oracle_b_matches_oracle_a_tiny_workload(oracle_lib):
    from paper_1912_12786_amd import workloads as W
    wl = W.tiny()
    n = _compare_a_b(oracle_lib, wl.vertices, wl.rays, "default", {})
    assert n == wl.n_rays  # no exception rays in this scene
    rng = np.random.default_rng(3)
    for kind in ("alpha", "procedural"):
        kw = _scene_params(rng, kind, wl.n_tris)
        assert _compare_a_b(oracle_lib, wl.vertices, wl.rays, kind, kw) > 0.95 * wl.n_rays


def test_any_hit_iff_closest_hit(oracle_lib):
    rng = np.random.default_rng(8)
    verts, rays = _random_scene(rng, 48, 512)
    for kind in ("default", "alpha", "procedural"):
        kw = _scene_params(rng, kind, verts.shape[0])
        bvh = oracle_lib.build_bvh(verts)
        c = oracle_lib.traverse(verts, bvh, rays, kind, **kw)
        a = oracle_lib.traverse(verts, bvh, rays, kind, any_hit=True, **kw)
        assert np.array_equal(c["prim"] == MISS, a["prim"] == MISS)
        # any-hit never tests more triangles than closest-hit needs... but its
        # stop is at the first accepted candidate, so it accepts exactly once
        hit = a["prim"] != MISS
        assert np.all(a["counters"][hit, 3] == 1)
        assert np.all(a["counters"][~hit, 3] == 0)
        ca = oracle_lib.brute(verts, rays, kind, **kw)
        ok = ca["flags"] == 0
        assert np.array_equal((ca["prim"] == MISS)[ok], (a["prim"] == MISS)[ok])


# ----------------------------------------------------------------------------
# counts against the order-free set formula
# ----------------------------------------------------------------------------
def _slab64(lo, hi, o, d, tmin, tmax):
    tiny = 2.0 ** -80
    dd = np.where(np.abs(d) < tiny, np.copysign(tiny, d), d)
    t0 = (lo - o) / dd
    t1 = (hi - o) / dd
    tn = max(np.max(np.minimum(t0, t1)), tmin)
    tf = min(np.min(np.maximum(t0, t1)), tmax)
    return tn, tf


def test_counts_without_accepts_follow_set_formula(oracle_lib):
    """With every candidate rejected, tmax never shrinks, so the visited set
    is independent of order: an inner node is entered iff its box and all its
    ancestors' boxes are hit.  Then boxes = 1 + 2 * (#entered inner nodes) and
    triangles = sum of the entered leaves' sizes."""
    from paper_1912_12786_amd import workloads as W
    wl = W.tiny()
    verts = wl.vertices
    n = verts.shape[0]
    tex = uniform_alpha_textures([0], (2, 2))
    kw = dict(geom_ids=np.zeros(n, np.uint32),
              texcoords=np.zeros((n, 3, 2), np.float32), textures=tex, alpha_min=1)
    bvh = oracle_lib.build_bvh(verts)
    rays = wl.rays[::7]
    B = oracle_lib.traverse(verts, bvh, rays, "alpha", **kw)
    assert np.all(B["prim"] == MISS) and np.all(B["counters"][:, 3] == 0)
    nodes = bvh.nodes
    lo = nodes["lo"].astype(np.float64)
    hi = nodes["hi"].astype(np.float64)
    checked = 0
    for i in range(rays.shape[0]):
        o = rays[i, :3].astype(np.float64)
        d = rays[i, 4:7].astype(np.float64)
        boxes, tris, grazing = 0, 0, False
        todo = [0]
        while todo:                      # set expansion, order irrelevant
            k = todo.pop()
            tn, tf = _slab64(lo[k], hi[k], o, d, 0.0, np.inf)
            if abs(tn - tf) <= 1e-5 * max(1.0, abs(tn)):
                grazing = True
            boxes += 1
            if tn > tf:
                continue
            if nodes["count"][k] > 0:
                tris += int(nodes["count"][k])
            else:
                todo += [int(nodes["left"][k]), int(nodes["right"][k])]
        if grazing:
            continue
        checked += 1
        assert B["counters"][i, 0] == boxes, i
        assert B["counters"][i, 1] == tris, i
    assert checked > 0.9 * rays.shape[0]


# ----------------------------------------------------------------------------
# builder pins
# ----------------------------------------------------------------------------
def _check_bvh_invariants(verts, bvh):
    nodes, perm = bvh.nodes, bvh.perm
    n = verts.shape[0]
    assert sorted(perm.tolist()) == list(range(n))
    tlo = verts.min(axis=1)
    thi = verts.max(axis=1)
    seen = np.zeros(n, np.int64)
    stack = [(0, 0)]
    order = []
    while stack:
        k, depth = stack.pop()
        order.append(k)
        nd = nodes[k]
        assert nd["depth"] == depth
        if nd["count"] > 0:
            assert nd["count"] <= 4
            idx = perm[nd["first"]:nd["first"] + nd["count"]]
            seen[idx] += 1
            assert np.array_equal(nd["lo"], tlo[idx].min(0)) and np.array_equal(nd["hi"], thi[idx].max(0))
        else:
            l, r = int(nd["left"]), int(nd["right"])
            assert l == k + 1            # preorder: left child follows its parent
            for c in (l, r):
                assert np.all(nodes[c]["lo"] >= nd["lo"]) and np.all(nodes[c]["hi"] <= nd["hi"])
            assert np.array_equal(nd["lo"], np.minimum(nodes[l]["lo"], nodes[r]["lo"]))
            assert np.array_equal(nd["hi"], np.maximum(nodes[l]["hi"], nodes[r]["hi"]))
            stack += [(r, depth + 1), (l, depth + 1)]
    assert order == sorted(order)        # visiting left-first reproduces preorder ids
    assert np.all(seen == 1)
    assert bvh.max_depth <= 64


def test_bvh_invariants_tiny_and_random(oracle_lib):
    from paper_1912_12786_amd import workloads as W
    _check_bvh_invariants(W.tiny().vertices, oracle_lib.build_bvh(W.tiny().vertices))
    rng = np.random.default_rng(2)
    for n in (1, 2, 4, 5, 9, 33, 300):
        v, _ = _random_scene(rng, n, 1)
        _check_bvh_invariants(v, oracle_lib.build_bvh(v))


def test_bvh_degenerate_centroids(oracle_lib):
    # identical triangles: no centroid extent anywhere -> index-median splits
    v = np.tile(np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0]]], np.float32), (37, 1, 1))
    bvh = oracle_lib.build_bvh(v)
    _check_bvh_invariants(v, bvh)
    assert bvh.nodes[0]["count"] == 0
    left = bvh.nodes[bvh.nodes[0]["left"]]
    assert left["count"] == 0 or left["count"] == 18


def _area(lo, hi):
    d = hi.astype(np.float64) - lo.astype(np.float64)
    return 2.0 * (d[0] * d[1] + d[1] * d[2] + d[2] * d[0])


def test_bvh_root_split_is_sah_minimum(oracle_lib):
    """The root's children are the minimum-cost binned split, enumerated here
    over all 3 x 31 candidate planes directly from the triangle boxes."""
    rng = np.random.default_rng(9)
    for trial in range(5):
        v, _ = _random_scene(rng, 200, 1)
        bvh = oracle_lib.build_bvh(v)
        tlo, thi = v.min(1), v.max(1)
        cen = 0.5 * (tlo.astype(np.float64) + thi.astype(np.float64))
        best = (np.inf, None)
        for a in range(3):
            cmin, cmax = cen[:, a].min(), cen[:, a].max()
            ext = cmax - cmin
            if ext <= 0:
                continue
            b = np.minimum(31, ((cen[:, a] - cmin) * (32.0 / ext)).astype(np.int64))
            for s in range(1, 32):
                L, R = b < s, b >= s
                if not L.any() or not R.any():
                    continue
                cost = (_area(tlo[L].min(0), thi[L].max(0)) * L.sum()
                        + _area(tlo[R].min(0), thi[R].max(0)) * R.sum())
                if cost < best[0]:
                    best = (cost, set(np.nonzero(L)[0].tolist()))
        left = bvh.nodes[bvh.nodes[0]["left"]]
        # the left child's triangles are the contiguous perm range before the right child's
        right = bvh.nodes[bvh.nodes[0]["right"]]
        first = min(left["first"], right["first"]) if left["count"] else 0
        # collect triangles under the left child
        stack, got = [int(bvh.nodes[0]["left"])], set()
        while stack:
            k = stack.pop()
            nd = bvh.nodes[k]
            if nd["count"] > 0:
                got |= set(bvh.perm[nd["first"]:nd["first"] + nd["count"]].tolist())
            else:
                stack += [int(nd["left"]), int(nd["right"])]
        assert got == best[1], trial
        del first


def test_bvh_deterministic(oracle_lib):
    from paper_1912_12786_amd import workloads as W
    v = W.tiny().vertices
    a, b = oracle_lib.build_bvh(v), oracle_lib.build_bvh(v)
    assert a.nodes.tobytes() == b.nodes.tobytes() and np.array_equal(a.perm, b.perm)


# ----------------------------------------------------------------------------
# leaf size limit of the build
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("max_leaf", [1, 2, 3, 5, 7])
def test_bvh_leaf_limit(oracle_lib, max_leaf):
    """Leaves hold at most max_leaf triangles, inner nodes more; leaves
    partition the triangles; and the traversal still answers the float64
    definition (outside the exception set)."""
    rng = np.random.default_rng(20 + max_leaf)
    verts, rays = _random_scene(rng, 60, 300)
    bvh = oracle_lib.build_bvh(verts, max_leaf=max_leaf)
    nd = bvh.nodes
    leaves = nd[nd["count"] > 0]
    inner = nd[nd["count"] == 0]
    assert leaves["count"].max() <= max_leaf
    assert np.all(leaves["count"] >= 1)
    covered = np.zeros(60, int)
    for lf in leaves:
        covered[lf["first"]:lf["first"] + lf["count"]] += 1
    assert np.all(covered == 1)
    # an inner node's subtree holds more than max_leaf triangles
    def size(i):
        return int(nd[i]["count"]) if nd[i]["count"] else size(int(nd[i]["left"])) + size(int(nd[i]["right"]))
    assert all(size(i) > max_leaf for i in np.nonzero(nd["count"] == 0)[0])
    assert len(inner) == len(leaves) - 1
    for kind in ("default", "alpha"):
        kw = _scene_params(rng, kind, 60)
        A = oracle_lib.brute(verts, rays, kind, **kw)
        B = oracle_lib.traverse(verts, bvh, rays, kind, **kw)
        ok = A["flags"] == 0
        assert np.array_equal(A["prim"][ok], B["prim"][ok])


def test_root_leaf_counts_up_to_seven(oracle_lib):
    """A scene of N <= max_leaf triangles is one root leaf: every ray that
    hits the root box makes exactly 1 box test and N triangle tests (closest
    hit, accept-all), every other ray 1 box test and none."""
    rng = np.random.default_rng(8)
    for n in (5, 6, 7):
        verts, rays = _random_scene(rng, n, 400)
        bvh = oracle_lib.build_bvh(verts, max_leaf=7)
        assert bvh.n_nodes == 1 and bvh.nodes[0]["count"] == n
        B = oracle_lib.traverse(verts, bvh, rays)
        c = B["counters"]
        assert np.all(c[:, 0] == 1)
        assert set(np.unique(c[:, 1])) <= {0, n} and (c[:, 1] == n).sum() > 50
    with pytest.raises(ValueError):
        oracle_lib.build_bvh(verts, max_leaf=8)
