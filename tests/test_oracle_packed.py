"""Pins of oracle B's packed-reference (48-byte) node layout: child
references carried in the low bytes of child-box words moved outward (not in
the paper, whose node format is open).

The word move is checked against hand-derived cases (golden/packed_words.json)
and, on random floats, against the properties that define it: the carried
byte, the outward direction, no nearer pattern with that byte (the patterns
in between enumerated with integer arithmetic on value-ordered keys), and a
move of at most 255 patterns (511 for a walk across zero).  The packed BVH is checked for references that
gather back to the canonical ones (recomputed here from the node array), for
boxes that contain the canonical boxes, and the packed traversal against the
float64 definition (oracle A) and against the float32-box traversal."""
import json
import os

import numpy as np
import pytest

from tests.golden.load import HERE
from tests.test_oracle_pins import _random_scene, _scene_params

MISS = 0xFFFFFFFF


def _f(bits):
    return np.array([bits], np.uint32).view(np.float32)[0]


def _bits(x):
    return int(np.array([x], np.float32).view(np.uint32)[0])


def _key(bits):
    """Value-ordered key of a float32 pattern (-0 just below +0)."""
    return (~bits) & 0xFFFFFFFF if bits >> 31 else bits | 0x80000000


def _unkey(k):
    return k ^ 0x80000000 if k >= 0x80000000 else (~k) & 0xFFFFFFFF


with open(os.path.join(HERE, "packed_words.json")) as _fh:
    _GOLDEN = json.load(_fh)["cases"]


@pytest.mark.parametrize("case", _GOLDEN, ids=lambda c: f"{c['x']}-{c['byte']}-{c['lower']}")
def test_golden_word_moves(oracle_lib, case):
    got = oracle_lib.move_word(_f(int(case["x"], 16)), int(case["byte"], 16), case["lower"])
    if case["expect"] is None:
        assert got is None
    else:
        assert got is not None and _bits(got) == int(case["expect"], 16), case["why"]


def test_word_move_properties(oracle_lib):
    rng = np.random.default_rng(5)
    pats = np.concatenate([
        rng.integers(0, 2**32, 3000, dtype=np.uint64),              # any pattern
        rng.integers(0, 600, 300, dtype=np.uint64),                  # around +0
        0x80000000 + rng.integers(0, 600, 300, dtype=np.uint64),     # around -0
    ]).astype(np.uint32)
    checked = 0
    for p in pats:
        x = _f(int(p))
        if not np.isfinite(x):
            continue
        for lower in (True, False):
            byte = int(rng.integers(0, 256))
            y = oracle_lib.move_word(x, byte, lower)
            kx = _key(int(p))
            step = -1 if lower else 1
            # the nearest pattern outward carrying the byte, by key walk
            k = kx
            while (_unkey(k) & 0xFF) != byte:
                k += step
            want = _unkey(k)
            if not np.isfinite(_f(want)) or any(not np.isfinite(_f(_unkey(j)))
                                                for j in range(min(kx, k), max(kx, k) + 1)):
                assert y is None
                continue
            assert y is not None and _bits(y) == want
            assert (y <= x) if lower else (y >= x)
            # 255 patterns within one sign; a walk across zero restarts the
            # byte cycle on the other side
            crossed = (k < 0x80000000) != (kx < 0x80000000)
            assert abs(k - kx) <= (511 if crossed else 255)
            checked += 1
    assert checked > 5000


def _canonical_refs(nodes):
    """Child references of every inner node as the 64-byte layout stores
    them: an inner child's index among the inner nodes in preorder (the node
    array's order), a leaf child's count << 29 | first."""
    inner = np.cumsum(nodes["count"] == 0) - 1
    refs = np.zeros((len(nodes), 2), np.uint64)
    for n in range(len(nodes)):
        if nodes[n]["count"]:
            continue
        for c, ch in enumerate((nodes[n]["left"], nodes[n]["right"])):
            cnt = int(nodes[ch]["count"])
            refs[n, c] = (cnt << 29 | int(nodes[ch]["first"])) if cnt else int(inner[ch])
    return refs.astype(np.uint32)


@pytest.mark.parametrize("seed,n,max_leaf", [(1, 300, 4), (2, 2000, 2), (3, 17, 1), (4, 900, 7)])
def test_pack_references_and_boxes(oracle_lib, seed, n, max_leaf):
    rng = np.random.default_rng(seed)
    verts, _ = _random_scene(rng, n, 1)
    bvh = oracle_lib.build_bvh(verts, max_leaf=max_leaf)
    P = oracle_lib.pack(bvh)
    nodes, box, refs = bvh.nodes, P["box"], P["refs"]
    inner = nodes["count"] == 0
    assert np.array_equal(refs, _canonical_refs(nodes))
    w = box.view(np.uint32)
    for c in range(2):
        gathered = (w[:, 6*c] & 0xFF) | (w[:, 6*c+1] & 0xFF) << 8 | (w[:, 6*c+2] & 0xFF) << 16 \
            | (w[:, 6*c+3] & 0xFF) << 24
        assert np.array_equal(gathered[inner], refs[inner, c])
        child = np.where(c == 0, nodes["left"], nodes["right"])[inner]
        lo, hi = nodes["lo"][child], nodes["hi"][child]
        b = box[inner, 6*c:6*c+6]
        assert np.all(b[:, :3] <= lo) and np.all(b[:, 3:] >= hi)
        # hi.y and hi.z keep their canonical bits
        assert np.array_equal(b[:, 4:].view(np.uint32), hi[:, 1:].view(np.uint32))
    assert not box[~inner].any() and not refs[~inner].any()


@pytest.mark.parametrize("kind", ["default", "alpha", "procedural"])
@pytest.mark.parametrize("any_hit", [False, True])
def test_packed_traversal_matches_oracle_a(oracle_lib, kind, any_hit):
    for seed in range(6):
        rng = np.random.default_rng(100 + seed)
        n_tris = int(rng.integers(5, 80))
        verts, rays = _random_scene(rng, n_tris, 256)
        kw = _scene_params(rng, kind, n_tris)
        bvh = oracle_lib.build_bvh(verts, max_leaf=int(rng.integers(1, 5)))
        A = oracle_lib.brute(verts, rays, kind, any_hit=any_hit, **kw)
        B = oracle_lib.traverse(verts, bvh, rays, kind, any_hit=any_hit, layout="f32p", **kw)
        ok = A["flags"] == 0
        if any_hit:
            assert np.array_equal((A["prim"] == MISS)[ok], (B["prim"] == MISS)[ok])
            continue
        assert np.array_equal(A["prim"][ok], B["prim"][ok])
        hit = ok & (A["prim"] != MISS)
        tol_t = np.maximum(1e-5 * np.abs(A["t"][hit]), A["bound_t"][hit])
        assert np.all(np.abs(B["t"][hit] - A["t"][hit]) <= tol_t)


@pytest.mark.parametrize("kind", ["default", "alpha", "procedural"])
def test_packed_results_equal_f32_layout(oracle_lib, kind):
    """Without exact ties the moved words (supersets of the canonical boxes)
    change the counts but not the closest, any-hit or multi-hit answers."""
    rng = np.random.default_rng(78)
    verts, rays = _random_scene(rng, 400, 3000, size=(0.02, 0.1))
    kw = _scene_params(rng, kind, verts.shape[0])
    bvh = oracle_lib.build_bvh(verts, max_leaf=2)
    for extra in (dict(), dict(any_hit=True), dict(multi_k=3)):
        F = oracle_lib.traverse(verts, bvh, rays, kind, **extra, **kw)
        Pk = oracle_lib.traverse(verts, bvh, rays, kind, layout="f32p", **extra, **kw)
        if extra.get("any_hit"):
            assert np.array_equal(F["prim"] == MISS, Pk["prim"] == MISS)
            continue
        for k in ("prim", "t", "u", "v"):
            assert np.array_equal(np.asarray(F[k]).view(np.uint32), np.asarray(Pk[k]).view(np.uint32))
    F = oracle_lib.traverse(verts, bvh, rays, kind, **kw)
    Pk = oracle_lib.traverse(verts, bvh, rays, kind, layout="f32p", **kw)
    assert Pk["counters"][:, 0].sum() >= F["counters"][:, 0].sum()


def test_packed_traversal_tests_the_moved_words(oracle_lib):
    """Rays through the margin a moved lo word adds to a root child's box
    (inside the stored box, outside the canonical one): the packed traversal
    enters that child and box-tests its children, the float32 one does not."""
    rng = np.random.default_rng(11)
    verts, _ = _random_scene(rng, 3000, 1)
    bvh = oracle_lib.build_bvh(verts, max_leaf=2)
    nodes, box = bvh.nodes, oracle_lib.pack(bvh)["box"]
    root = nodes[0]
    rays = []
    for c, ch in enumerate((root["left"], root["right"])):
        if nodes[ch]["count"]:
            continue
        for a in range(3):
            L, Lp = np.float32(nodes[ch]["lo"][a]), box[0, 6 * c + a]
            xm = np.nextafter(L, np.float32(-np.inf))
            if not (Lp <= xm < L and L > root["lo"][a]):
                continue
            b, e = (a + 1) % 3, (a + 2) % 3
            o = np.zeros(3, np.float32)
            o[a] = xm
            o[b] = root["lo"][b] - 1.0
            o[e] = 0.5 * (nodes[ch]["lo"][e] + nodes[ch]["hi"][e])
            d = np.zeros(3, np.float32)
            d[b] = 1.0
            rays.append([*o, 0.0, *d, 100.0])
    assert len(rays) >= 2
    rays = np.asarray(rays, np.float32)
    F = oracle_lib.traverse(verts, bvh, rays)
    Pk = oracle_lib.traverse(verts, bvh, rays, layout="f32p")
    assert np.all(Pk["counters"][:, 0] >= F["counters"][:, 0] + 2)


def test_packed_root_leaf_counts(oracle_lib):
    """A root leaf has no inner node to pack: counts as for float32 boxes."""
    rng = np.random.default_rng(3)
    verts, rays = _random_scene(rng, 4, 300)
    bvh = oracle_lib.build_bvh(verts)
    assert bvh.nodes[0]["count"] == 4
    F = oracle_lib.traverse(verts, bvh, rays)
    Pk = oracle_lib.traverse(verts, bvh, rays, layout="f32p")
    assert np.array_equal(F["counters"], Pk["counters"])


def test_packed_empty_scene(oracle_lib):
    """No triangles: nothing to pack, every ray misses with no box test."""
    bvh = oracle_lib.build_bvh(np.zeros((0, 3, 3), np.float32))
    P = oracle_lib.pack(bvh)
    assert not P["box"].any() and not P["refs"].any()
    rays = np.zeros((5, 8), np.float32)
    rays[:, 6], rays[:, 7] = -1.0, np.inf
    B = oracle_lib.traverse(np.zeros((0, 3, 3), np.float32), bvh, rays, layout="f32p")
    assert np.all(B["prim"] == MISS) and not B["counters"].any()
