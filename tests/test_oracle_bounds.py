"""Pins of oracle A's float32 error bounds and exception-set flags.

Oracle A (the float64 definition of the closest hit, Section 3.1) reports per
ray an a-priori forward-error bound of a float32 ray/triangle test, ``B_uv``
and ``B_t``, and flags rays whose answer is fragile (near ties, hits near a
triangle edge, accept decisions of the alpha mask of Section 4 or of the
procedural checker near their boundary).  Both decide how the float32 results
are compared with the float64 definition, so both are pinned here against
things other than the oracle's own formulas:

* the bounds against actual float32 evaluations: oracle B's fused
  Moller-Trumbore (the operation sequence the GPU follows bit for bit) and an
  independent unfused numpy float32 evaluation, on far, near, grazing and
  instanced hits -- never exceeded, and never vacuous (the worst observed
  error is a stated fraction of the bound);
* the flags on constructed hits at, and 0.1 texel or cell away from, a texel
  edge whose two sides decide differently, a texel edge whose two sides decide
  alike, and a checker line.
"""
import numpy as np
import pytest

from paper_1912_12786_amd import workloads as W

MISS = 0xFFFFFFFF

# The bounds are worst-case sums of norms (Cauchy-Schwarz on every product), so
# they sit above the largest error ever seen; they must not sit so far above it
# that a comparison against them checks nothing.  Observed worst-error / bound
# ratios on the scenes below: u/v 0.03-0.08, t 0.11-0.15.
MIN_WORST_RATIO = 1e-2


def _mt32_numpy(verts, rays, prim):
    """Unfused float32 Moller-Trumbore of each ray against triangle ``prim``
    (numpy rounds every operation to float32; no fused multiply-add)."""
    f = np.float32
    tri = np.asarray(verts, f).reshape(-1, 3, 3)[prim]
    r = np.asarray(rays, f)
    o, d = r[:, 0:3], r[:, 4:7]
    e1 = tri[:, 1] - tri[:, 0]
    e2 = tri[:, 2] - tri[:, 0]
    s = o - tri[:, 0]

    def cross(a, b):
        return np.stack([a[:, 1] * b[:, 2] - a[:, 2] * b[:, 1],
                         a[:, 2] * b[:, 0] - a[:, 0] * b[:, 2],
                         a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0]], axis=1)

    def dot(a, b):
        return (a[:, 0] * b[:, 0] + a[:, 1] * b[:, 1]) + a[:, 2] * b[:, 2]

    p = cross(d, e2)
    det = dot(e1, p)
    rr = f(1) / det
    u = dot(s, p) * rr
    q = cross(s, e1)
    v = dot(d, q) * rr
    t = dot(e2, q) * rr
    return t, u, v


def _errors_within_bounds(A, t, u, v, sel, what):
    dt = np.abs(t[sel].astype(np.float64) - A["t"][sel])
    du = np.abs(u[sel].astype(np.float64) - A["u"][sel])
    dv = np.abs(v[sel].astype(np.float64) - A["v"][sel])
    bt, bu = A["bound_t"][sel], A["bound_uv"][sel]
    assert np.all(dt <= bt), f"{what}: |dt| above B_t on {(dt > bt).sum()} rays"
    assert np.all(du <= bu), f"{what}: |du| above B_uv on {(du > bu).sum()} rays"
    assert np.all(dv <= bu), f"{what}: |dv| above B_uv on {(dv > bu).sum()} rays"
    return float((np.maximum(du, dv) / bu).max()), float((dt / bt).max())


def _grazing_scene(seed, n_tris=400, n_rays=3000):
    """Unit-size triangles near the origin seen at shallow angles (|cos| down
    to about 0.02), from distances 1..50: ill-conditioned tests."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-1, 1, size=(n_tris, 1, 3))
    nrm = np.tile(np.array([0.0, 0.0, 1.0]), (n_tris, 1))
    a = np.cross(nrm, rng.normal(size=(n_tris, 3)))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = np.cross(nrm, a)
    ang = rng.uniform(0, 2 * np.pi, size=(n_tris, 1)) + 2 * np.pi * np.arange(3) / 3
    verts = c + 0.3 * (np.cos(ang)[..., None] * a[:, None] + np.sin(ang)[..., None] * b[:, None])
    verts = verts.astype(np.float32)
    target = rng.uniform(-1, 1, size=(n_rays, 3)) * [1, 1, 0]
    elev = rng.uniform(0.02, 0.5, size=n_rays)
    az = rng.uniform(0, 2 * np.pi, size=n_rays)
    dirn = np.stack([np.cos(az) * np.cos(elev), np.sin(az) * np.cos(elev), -np.sin(elev)], 1)
    dist = rng.uniform(1, 50, size=(n_rays, 1))
    rays = np.zeros((n_rays, 8), np.float32)
    rays[:, 0:3] = target - dist * dirn
    rays[:, 4:7] = dirn
    rays[:, 7] = np.inf
    return verts, rays


def _scenes():
    wl = W.tiny()
    yield "tiny 1,024 triangles", wl.vertices, wl.rays
    bb = W.billboards(n_quads=3000, width=160, height=90)
    yield "billboards at distance 60-160", bb.vertices, bb.rays
    sp = W.spheres(n_spheres=60, width=160, height=90)
    yield "tessellated spheres", sp.vertices, sp.rays
    gv, gr = _grazing_scene(5)
    yield "grazing hits", gv, gr


@pytest.mark.parametrize("case", range(4))
def test_float32_error_bounds_hold_and_are_not_vacuous(oracle_lib, case):
    name, verts, rays = list(_scenes())[case]
    A = oracle_lib.brute(verts, rays)
    B = oracle_lib.traverse(verts, oracle_lib.build_bvh(verts), rays)
    hit = (A["prim"] != MISS) & (A["flags"] == 0) & (B["prim"] == A["prim"])
    assert hit.sum() >= 300, f"{name}: too few clean hits ({hit.sum()}) to judge the bound"
    ruv, rt = _errors_within_bounds(A, B["t"], B["u"], B["v"], hit, f"{name}, fused float32")
    assert ruv >= MIN_WORST_RATIO, f"{name}: B_uv is {1 / ruv:.0f}x the worst u/v error"
    assert rt >= MIN_WORST_RATIO, f"{name}: B_t is {1 / rt:.0f}x the worst t error"
    # a second float32 evaluation with a different operation order
    prim = np.where(A["prim"] == MISS, 0, A["prim"]).astype(np.int64)
    t, u, v = _mt32_numpy(verts, rays, prim)
    _errors_within_bounds(A, t, u, v, hit, f"{name}, unfused float32")


def test_tiny_scene_tolerance_widening(oracle_lib):
    """On the tiny scene (triangles of side 0.05 seen from distance 2), the
    float32 test's u/v error can exceed the benchmark spec's figure of 1e-5: the
    a-priori bound exceeds 1e-5 on every hit ray (median about 8e-5), so the
    comparison uses max(1e-5, B_uv).  The t bound exceeds 1e-5 t on a few
    percent of hits.  Actual errors above 1e-5 are rare."""
    wl = W.tiny()
    A = oracle_lib.brute(wl.vertices, wl.rays)
    B = oracle_lib.traverse(wl.vertices, oracle_lib.build_bvh(wl.vertices), wl.rays)
    hit = (A["prim"] != MISS) & (A["flags"] == 0) & (B["prim"] == A["prim"])
    n = int(hit.sum())
    frac_uv = float((A["bound_uv"][hit] > 1e-5).mean())
    frac_t = float((A["bound_t"][hit] > 1e-5 * A["t"][hit]).mean())
    med = float(np.median(A["bound_uv"][hit]))
    assert frac_uv == 1.0 and 3e-5 < med < 2e-4, (frac_uv, med)
    assert frac_t < 0.05, frac_t
    duv = np.maximum(np.abs(B["u"][hit] - A["u"][hit]), np.abs(B["v"][hit] - A["v"][hit]))
    over = int((duv > 1e-5).sum())
    assert over <= max(2, n // 200), f"{over} of {n} hits have a u/v error above 1e-5"
    dt = np.abs(B["t"][hit] - A["t"][hit])
    assert np.all(dt <= 1e-5 * A["t"][hit]), "a t error above 1e-5 relative on the tiny scene"


# ----------------------------------------------------------------------------
# exception flags on constructed hits
# ----------------------------------------------------------------------------
# A unit quad at z = 0 split along its diagonal, texture coordinates equal to
# (x, y): triangle 0 = (0,0),(1,0),(1,1), triangle 1 = (0,0),(1,1),(0,1).  A
# ray straight down at (x, y) with y < x hits triangle 0 with u = x - y,
# v = y, so the interpolated texture coordinate is exactly (s, t) = (x, y)
# and lands on texel (floor(16 x), floor(16 y)) of a 16 x 16 texture.
QUAD = np.array([[[0, 0, 0], [1, 0, 0], [1, 1, 0]],
                 [[0, 0, 0], [1, 1, 0], [0, 1, 0]]], np.float32)
QUAD_TC = np.array([[[0, 0], [1, 0], [1, 1]],
                    [[0, 0], [1, 1], [0, 1]]], np.float32)
TEX = 16
TEXEL = 1.0 / TEX


def _down_rays(xy):
    r = np.zeros((len(xy), 8), np.float32)
    r[:, 0:2] = np.asarray(xy, np.float64)
    r[:, 2] = 1.0
    r[:, 6] = -1.0
    r[:, 7] = np.inf
    return r


def _split_texture(axis):
    """Opaque where texel x < 8 (axis 0) or texel y < 4 (axis 1), transparent
    elsewhere: the accept decision changes at s = 0.5, or at t = 0.25."""
    yy, xx = np.mgrid[0:TEX, 0:TEX]
    opaque = (xx < 8) if axis == 0 else (yy < 4)
    return np.where(opaque, 0xFF000000, 0x00FFFFFF).astype(np.uint32)[None]


# (x, y, texel-edge case, expect NEAR_FILTER, expected prim)
ALPHA_CASES_S = [
    (0.5, 0.2, "on the deciding edge s = 1/2", True, MISS),
    (0.5 + 1e-6, 0.2, "1e-6 past the deciding edge", True, MISS),
    (0.5 - 1e-6, 0.2, "1e-6 before the deciding edge", True, 0),
    (0.5 + 0.1 * TEXEL, 0.2, "0.1 texel past the deciding edge", False, MISS),
    (0.5 - 0.1 * TEXEL, 0.2, "0.1 texel before the deciding edge", False, 0),
    (0.25, 0.2 + 0.3 * TEXEL, "on an edge between two opaque texels", False, 0),
    (0.75, 0.2 + 0.3 * TEXEL, "on an edge between two clear texels", False, MISS),
]
ALPHA_CASES_T = [
    (0.6, 0.25, "on the deciding edge t = 1/4", True, MISS),
    (0.6, 0.25 - 1e-6, "1e-6 before the deciding edge", True, 0),
    (0.6, 0.25 - 0.1 * TEXEL, "0.1 texel before the deciding edge", False, 0),
    (0.6, 0.25 + 0.1 * TEXEL, "0.1 texel past the deciding edge", False, MISS),
    (0.6 + 0.3 * TEXEL, 0.125, "on an edge between two opaque texels", False, 0),
]


@pytest.mark.parametrize("axis,cases", [(0, ALPHA_CASES_S), (1, ALPHA_CASES_T)])
def test_alpha_near_filter_flag(oracle_lib, axis, cases):
    tex = _split_texture(axis)
    rays = _down_rays([(x, y) for x, y, *_ in cases])
    geom = np.zeros(2, np.uint32)
    kw = dict(geom_ids=geom, texcoords=QUAD_TC, textures=tex, alpha_min=128)
    A = oracle_lib.brute(QUAD, rays, "alpha", **kw)
    M = oracle_lib.brute_multi(QUAD, rays, 2, "alpha", **kw)
    for i, (x, y, what, flagged, prim) in enumerate(cases):
        got = bool(A["flags"][i] & oracle_lib.E_NEAR_FILTER)
        assert got == flagged, f"closest hit, {what}: NEAR_FILTER {got}"
        assert not A["flags"][i] & oracle_lib.E_NEAR_EDGE, what
        assert A["prim"][i] == prim, f"{what}: prim {A['prim'][i]}"
        got_m = bool(M["flags"][i] & oracle_lib.E_NEAR_FILTER)
        assert got_m == flagged, f"multi-hit, {what}: NEAR_FILTER {got_m}"
    # the same quad as one instance under the identity map
    ident = np.array([[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]], np.float32)
    I = oracle_lib.brute_instanced([QUAD], [0], ident, rays, "alpha", geom_ids=[geom],
                                   texcoords=[QUAD_TC], textures=tex, alpha_min=128)
    for i, (x, y, what, flagged, prim) in enumerate(cases):
        got = bool(I["flags"][i] & oracle_lib.E_NEAR_FILTER)
        assert got == flagged, f"instanced, {what}: NEAR_FILTER {got}"


# Triangle (0,0,0),(1,0,0),(0,1,0) seen straight down: u = x, v = y.  The
# checker with n = 8 changes its decision where 8u or 8v is an integer.
CHECKER_TRI = np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0]]], np.float32)
CELL = 1.0 / 8
CHECKER_CASES = [
    (0.25, 0.1, "on the line 8u = 2", True),
    (0.25 + 1e-7, 0.1, "1e-7 past the line 8u = 2", True),
    (0.25 + 0.1 * CELL, 0.1, "0.1 cell past the line 8u = 2", False),
    (0.25 - 0.1 * CELL, 0.1, "0.1 cell before the line 8u = 2", False),
    (0.1, 0.375, "on the line 8v = 3", True),
    (0.1, 0.375 + 0.1 * CELL, "0.1 cell past the line 8v = 3", False),
    (0.3, 0.3, "0.4 cell from every line", False),
]


def test_checker_near_filter_flag(oracle_lib):
    rays = _down_rays([(x, y) for x, y, *_ in CHECKER_CASES])
    A = oracle_lib.brute(CHECKER_TRI, rays, "procedural", checker_n=8)
    M = oracle_lib.brute_multi(CHECKER_TRI, rays, 2, "procedural", checker_n=8)
    ident = np.array([[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]], np.float32)
    I = oracle_lib.brute_instanced([CHECKER_TRI], [0], ident, rays, "procedural", checker_n=8)
    for i, (x, y, what, flagged) in enumerate(CHECKER_CASES):
        for name, R in (("closest", A), ("multi-hit", M), ("instanced", I)):
            got = bool(R["flags"][i] & oracle_lib.E_NEAR_FILTER)
            assert got == flagged, f"{name}, {what}: NEAR_FILTER {got}"
        accept = (int(np.floor(8 * x)) + int(np.floor(8 * y))) % 2 == 0
        if not flagged:
            assert (A["prim"][i] == 0) == accept, what


def test_default_intersector_never_flags_filter(oracle_lib):
    rays = _down_rays([(x, y) for x, y, *_ in CHECKER_CASES])
    A = oracle_lib.brute(CHECKER_TRI, rays)
    assert not np.any(A["flags"] & oracle_lib.E_NEAR_FILTER)


def test_near_edge_flag_distance(oracle_lib):
    """NEAR_EDGE marks hits whose edge margin min(u, v, 1-u-v) is under
    max(1e-6, B_uv): 1e-7 from the edge v = 0 is flagged, 1e-3 is not."""
    rays = _down_rays([(0.3, 0.0), (0.3, 1e-7), (0.3, 1e-3), (0.3, 0.3)])
    A = oracle_lib.brute(CHECKER_TRI, rays)
    got = [bool(f & oracle_lib.E_NEAR_EDGE) for f in A["flags"]]
    assert got == [True, True, False, False], got
    assert np.all(A["bound_uv"] < 1e-5) and np.all(A["bound_uv"] > 1e-7)


# ----------------------------------------------------------------------------
# instanced hits: the bound adds the object-ray transform's rounding
# ----------------------------------------------------------------------------
def _instanced_scene(seed, n_inst=40, n_rays=4000, offset=0.0):
    rng = np.random.default_rng(seed)
    mesh = W.uv_sphere(np.zeros(3), 1.0).astype(np.float32)
    m = np.zeros((n_inst, 12), np.float32)
    pos = rng.uniform(0, 100, size=(n_inst, 3)) + offset
    scale = rng.uniform(0.3, 3.0, size=n_inst)
    for j in range(n_inst):
        q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        inv = np.linalg.inv(scale[j] * q)
        m[j, [0, 1, 2, 4, 5, 6, 8, 9, 10]] = inv.reshape(-1)
        m[j, [3, 7, 11]] = -inv @ pos[j]
    eye = np.array([50.0, 50.0, -80.0]) + offset
    # aim every ray at a point inside a random instance's sphere
    j = rng.integers(0, n_inst, size=n_rays)
    tgt = pos[j] + 0.8 * scale[j, None] * rng.uniform(-0.57, 0.57, size=(n_rays, 3))
    d = tgt - eye
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.zeros((n_rays, 8), np.float32)
    rays[:, 0:3] = eye
    rays[:, 4:7] = d
    rays[:, 7] = np.inf
    return mesh, m, rays


@pytest.mark.parametrize("offset", [0.0, 2e4])
def test_instanced_float32_error_bounds(oracle_lib, offset):
    """Instances rotated, scaled 0.3-3x and translated within a box of side
    100, itself moved ``offset`` from the origin with the eye: far from the
    origin the object-space ray's rounding (its terms are about ``offset``
    while it is about 100) outweighs the triangle test's own, and the
    instanced bound must carry it."""
    mesh, m, rays = _instanced_scene(11, offset=offset)
    n_inst = m.shape[0]
    bvh = oracle_lib.build_bvh(mesh)
    # world boxes of the transformed unit sphere (radius times scale, padded)
    lin = np.zeros((n_inst, 3, 3))
    lin[:] = m[:, [0, 1, 2, 4, 5, 6, 8, 9, 10]].reshape(-1, 3, 3)
    wfo = np.linalg.inv(lin)
    centre = np.einsum("nij,nj->ni", wfo, -m[:, [3, 7, 11]].astype(np.float64))
    rad = np.linalg.norm(wfo, ord=2, axis=(1, 2)) * 1.01
    tlas = oracle_lib.build_tlas(centre - rad[:, None], centre + rad[:, None])
    ids = np.zeros(n_inst, np.uint32)
    A = oracle_lib.brute_instanced([mesh], ids, m, rays)
    B = oracle_lib.traverse_instanced([mesh], [bvh], ids, m, tlas, rays)
    hit = ((A["prim"] != MISS) & (A["flags"] == 0) & (B["prim"] == A["prim"]) &
           (B["inst"] == A["inst"]))
    assert hit.sum() >= 300, hit.sum()
    ruv, rt = _errors_within_bounds(A, B["t"], B["u"], B["v"], hit, "instanced")
    assert ruv >= MIN_WORST_RATIO and rt >= MIN_WORST_RATIO, (ruv, rt)
