"""Pins of oracle B's 32-byte node layout (8-bit child boxes on a per-node
frame; not in the paper, whose BVH format is open).

The quantizer is checked against the properties that define it -- the
decoded box contains the exact box, no tighter 8-bit value would, the scale
exponent is the smallest that reaches the frame's far side, the origin is the
largest admissible float below the frame -- using exact rational arithmetic
for every fused multiply-add, and against two nodes derived by hand
(golden/q8_nodes.json).  The compressed traversal is checked against the
float64 definition (oracle A) and against the float32-box traversal."""
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from tests.golden.load import HERE
from tests.test_oracle_pins import _random_scene, _scene_params

MISS = 0xFFFFFFFF


# ----------------------------------------------------------------------------
# exact float32 arithmetic
# ----------------------------------------------------------------------------
def round_f32(x: Fraction) -> float:
    """x rounded to the nearest float32 (ties to even), normal range only."""
    if x == 0:
        return 0.0
    sign = -1 if x < 0 else 1
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    assert -126 <= e <= 127, "outside the normal float32 range"
    scaled = a / Fraction(2) ** (e - 23)          # in [2^23, 2^24)
    m = scaled.numerator // scaled.denominator
    rem = scaled - m
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and m % 2 == 1):
        m += 1
    return float(np.float32(sign * m * 2.0 ** (e - 23)))


def fma_f32(a, b, c) -> float:
    return round_f32(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


def f32_of_bits(b: int) -> float:
    return float(np.array([b], np.uint32).view(np.float32)[0])


def bits_of_f32(f: float) -> int:
    return int(np.array([f], np.float32).view(np.uint32)[0])


def frame_parts(F: int):
    return f32_of_bits(F & ~0xFF), 2.0 ** ((F & 0xFF) - 127), F & 0xFF


def decode(q: int, F: int) -> float:
    org, s, _ = frame_parts(F)
    return fma_f32(q, s, org)


def child_boxes(bvh, n):
    nd = bvh.nodes[n]
    return [(bvh.nodes[int(nd["left"])]["lo"], bvh.nodes[int(nd["left"])]["hi"]),
            (bvh.nodes[int(nd["right"])]["lo"], bvh.nodes[int(nd["right"])]["hi"])]


def check_node(bvh, Q, n):
    """Every defining property of node n's frame words and 8-bit values."""
    boxes = child_boxes(bvh, n)
    for a in range(3):
        F = int(Q["frames"][n, a])
        org, s, E = frame_parts(F)
        L = min(float(boxes[0][0][a]), float(boxes[1][0][a]))
        H = max(float(boxes[0][1][a]), float(boxes[1][1][a]))
        # origin: admissible pattern, below the frame, the largest such
        assert 1 <= E <= 254
        assert org <= L
        ob = bits_of_f32(org)
        nxt = f32_of_bits(ob - 0x100) if org < 0 else f32_of_bits(ob + 0x100)
        if org != 0 or ob == 0:
            assert nxt > L
        # scale: reaches H, and the next smaller one does not
        assert fma_f32(255, s, org) >= H
        if E > 1:
            assert fma_f32(255, s / 2, org) < H
        for c in range(2):
            lo, hi = float(boxes[c][0][a]), float(boxes[c][1][a])
            qlo = int(Q["q"][n, 6 * c + a])
            qhi = int(Q["q"][n, 6 * c + 3 + a])
            dlo, dhi = decode(qlo, F), decode(qhi, F)
            assert dlo <= lo and dhi >= hi                       # conservative
            if qlo < 255:
                assert decode(qlo + 1, F) > lo                   # tightest
            if qhi > 0:
                assert decode(qhi - 1, F) < hi
            assert Q["qbox"][n, 6 * c + a] == np.float32(dlo)    # decode as stored
            assert Q["qbox"][n, 6 * c + 3 + a] == np.float32(dhi)


def test_round_f32_against_numpy():
    rng = np.random.default_rng(0)
    for x in rng.normal(0, 1e3, size=200):
        assert round_f32(Fraction(float(x))) == float(np.float32(x))
    # ties to even: 1 + 2^-24 lies halfway between 1 and 1 + 2^-23
    assert round_f32(Fraction(1) + Fraction(1, 2 ** 24)) == 1.0
    assert round_f32(Fraction(1) + Fraction(3, 2 ** 24)) == 1.0 + 2.0 ** -22


# ----------------------------------------------------------------------------
# hand-derived nodes
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["positive", "negative"])
def test_golden_q8_nodes(oracle_lib, case):
    import json
    import os
    with open(os.path.join(HERE, "q8_nodes.json")) as f:
        fx = json.load(f)["cases"][case]
    verts = np.asarray(fx["vertices"], np.float32)
    bvh = oracle_lib.build_bvh(verts)
    root = bvh.nodes[0]
    assert root["count"] == 0
    left, right = bvh.nodes[int(root["left"])], bvh.nodes[int(root["right"])]
    assert (int(left["count"]), int(right["count"])) == (3, 2)
    Q = oracle_lib.quantize(bvh)
    assert Q["frames"][0].tolist() == fx["frames"]
    assert Q["q"][0].tolist() == fx["q"]
    check_node(bvh, Q, 0)


# ----------------------------------------------------------------------------
# properties on random scenes of several scales
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("seed,scale,shift,flat", [
    (1, 1.0, 0.0, False), (2, 100.0, 0.0, False), (3, 1.0, -0.5, False),
    (4, 1e-3, 7.0, False), (5, 50.0, -80.0, True), (6, 1e4, 1e4, False)])
def test_quantize_properties(oracle_lib, seed, scale, shift, flat):
    rng = np.random.default_rng(seed)
    verts, _ = _random_scene(rng, 60, 1)
    verts = (verts.astype(np.float64) * scale + shift).astype(np.float32)
    if flat:  # axis-aligned flat triangles: zero-extent boxes on one axis
        verts[::2, :, 2] = verts[::2, :1, 2]
    bvh = oracle_lib.build_bvh(verts)
    Q = oracle_lib.quantize(bvh)
    inner = np.nonzero(bvh.nodes["count"] == 0)[0]
    assert inner.size > 5
    for n in inner:
        check_node(bvh, Q, int(n))
    assert not Q["q"][bvh.nodes["count"] > 0].any()


# ----------------------------------------------------------------------------
# the compressed traversal
# ----------------------------------------------------------------------------
@settings(max_examples=25, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), n_tris=st.integers(5, 64),
       kind=st.sampled_from(["default", "alpha", "procedural"]), any_hit=st.booleans())
def test_q8_traversal_matches_oracle_a(oracle_lib, seed, n_tris, kind, any_hit):
    rng = np.random.default_rng(seed)
    verts, rays = _random_scene(rng, n_tris, 256)
    kw = _scene_params(rng, kind, n_tris)
    bvh = oracle_lib.build_bvh(verts)
    A = oracle_lib.brute(verts, rays, kind, any_hit=any_hit, **kw)
    B = oracle_lib.traverse(verts, bvh, rays, kind, any_hit=any_hit, layout="q8", **kw)
    ok = A["flags"] == 0
    if any_hit:
        assert np.array_equal((A["prim"] == MISS)[ok], (B["prim"] == MISS)[ok])
        return
    assert np.array_equal(A["prim"][ok], B["prim"][ok])
    hit = ok & (A["prim"] != MISS)
    tol_t = np.maximum(1e-5 * np.abs(A["t"][hit]), A["bound_t"][hit])
    assert np.all(np.abs(B["t"][hit] - A["t"][hit]) <= tol_t)


@pytest.mark.parametrize("kind", ["default", "alpha", "procedural"])
def test_q8_results_equal_f32_layout(oracle_lib, kind):
    """Without exact ties the decoded boxes (supersets) change the counts but
    not the closest, any-hit or multi-hit answers."""
    rng = np.random.default_rng(77)
    verts, rays = _random_scene(rng, 400, 3000, size=(0.02, 0.1))
    kw = _scene_params(rng, kind, verts.shape[0])
    bvh = oracle_lib.build_bvh(verts)
    for extra in (dict(), dict(any_hit=True), dict(multi_k=3)):
        F = oracle_lib.traverse(verts, bvh, rays, kind, **extra, **kw)
        Qd = oracle_lib.traverse(verts, bvh, rays, kind, layout="q8", **extra, **kw)
        if extra.get("any_hit"):
            assert np.array_equal(F["prim"] == MISS, Qd["prim"] == MISS)
            continue
        for k in ("prim", "t", "u", "v"):
            assert np.array_equal(np.asarray(F[k]).view(np.uint32), np.asarray(Qd[k]).view(np.uint32))
    # looser boxes: never fewer box tests in total, and some more
    F = oracle_lib.traverse(verts, bvh, rays, kind, **kw)
    Qd = oracle_lib.traverse(verts, bvh, rays, kind, layout="q8", **kw)
    assert Qd["counters"][:, 0].sum() > F["counters"][:, 0].sum()


def test_q8_root_leaf_counts(oracle_lib):
    """A root leaf has no quantized node: counts (1, N) as for float32 boxes."""
    rng = np.random.default_rng(3)
    verts, rays = _random_scene(rng, 4, 300)
    bvh = oracle_lib.build_bvh(verts)
    assert bvh.nodes[0]["count"] == 4
    F = oracle_lib.traverse(verts, bvh, rays)
    Qd = oracle_lib.traverse(verts, bvh, rays, layout="q8")
    assert np.array_equal(F["counters"], Qd["counters"])
    assert set(np.unique(F["counters"][:, 1])) <= {0, 4}
