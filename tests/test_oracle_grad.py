"""Pins of the oracle's hit gradient (float64 closed form from implicit
differentiation of o + t d = (1-u-v) v0 + u v1 + v v2) against central finite
differences of (t, u, v) recomputed with LAPACK (numpy.linalg.solve), and of
its fixed-prim (t, u, v) against the same solves."""
import numpy as np

from paper_1912_12786_amd import workloads as W


def solve_tuv(o, d, v0, v1, v2):
    M = np.stack([d, -(v1 - v0), -(v2 - v0)], axis=-1)
    return np.linalg.solve(M, (v0 - o)[..., None])[..., 0]


def small_mesh(seed=0):
    v, f = W.geodesic_sphere(4)
    rng = np.random.default_rng(seed)
    v = (v + rng.normal(0, 0.01, size=v.shape)).astype(np.float32)
    return v, f.astype(np.uint32)


def rays_at_faces(v, f, prims, rng):
    """Rays from outside aimed at interior points of the given faces."""
    tri = v[f[prims]].astype(np.float64)
    b = rng.dirichlet([2.0, 2.0, 2.0], size=len(prims))
    p = np.einsum("nk,nkj->nj", b, tri)
    o = p * 3.0 + rng.normal(0, 0.1, size=p.shape)
    d = p - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = np.zeros((len(prims), 8), np.float32)
    r[:, :3] = o
    r[:, 4:7] = d
    r[:, 7] = np.inf
    return r


def test_fixed_hit64_matches_lapack(oracle_lib):
    rng = np.random.default_rng(1)
    v, f = small_mesh()
    prims = rng.integers(0, f.shape[0], size=200).astype(np.uint32)
    rays = rays_at_faces(v, f, prims, rng)
    tuv = oracle_lib.fixed_hit64(v.astype(np.float64), f, rays, prims)
    tri = v[f[prims]].astype(np.float64)
    ref = solve_tuv(rays[:, :3].astype(np.float64), rays[:, 4:7].astype(np.float64),
                    tri[:, 0], tri[:, 1], tri[:, 2])
    assert np.allclose(tuv, ref, rtol=1e-10, atol=1e-12)
    miss = oracle_lib.fixed_hit64(v.astype(np.float64), f, rays[:1],
                                  np.array([oracle_lib.MISS], np.uint32))
    assert np.all(np.isnan(miss))


def test_hit_grad64_matches_central_differences(oracle_lib):
    rng = np.random.default_rng(2)
    v, f = small_mesh(3)
    v64 = v.astype(np.float64)
    prims = rng.integers(0, f.shape[0], size=300).astype(np.uint32)
    rays = rays_at_faces(v, f, prims, rng)
    g = rng.uniform(-1, 1, size=(len(prims), 3))
    gv, gr = oracle_lib.hit_grad64(v64, f, rays, prims, g)
    o = rays[:, :3].astype(np.float64)
    d = rays[:, 4:7].astype(np.float64)

    def loss(vv, oo=o, dd=d):
        tri = vv[f[prims]]
        return float(np.sum(g * solve_tuv(oo, dd, tri[:, 0], tri[:, 1], tri[:, 2])))

    h = 1e-4
    touched = np.unique(f[prims])
    for vid in rng.choice(touched, size=25, replace=False):
        for k in range(3):
            vp, vm = v64.copy(), v64.copy()
            vp[vid, k] += h
            vm[vid, k] -= h
            fd = (loss(vp) - loss(vm)) / (2 * h)
            assert abs(fd - gv[vid, k]) <= 1e-6 * max(1.0, abs(fd)), (vid, k, fd, gv[vid, k])
    # ray gradients: perturb one ray's origin / direction
    for i in rng.choice(len(prims), size=10, replace=False):
        for k in range(3):
            for which, arr in ((0, o), (3, d)):
                ap, am = arr.copy(), arr.copy()
                ap[i, k] += h
                am[i, k] -= h
                lp = loss(v64, ap, d) if which == 0 else loss(v64, o, ap)
                lm = loss(v64, am, d) if which == 0 else loss(v64, o, am)
                fd = (lp - lm) / (2 * h)
                assert abs(fd - gr[i, which + k]) <= 1e-6 * max(1.0, abs(fd))
    # vertices no ray touches get no gradient
    untouched = np.setdiff1d(np.arange(v.shape[0]), touched)
    assert np.all(gv[untouched] == 0)


def test_hit_grad64_closed_form_on_axis_aligned_triangle(oracle_lib):
    # triangle (0,0,0),(1,0,0),(0,1,0), ray down the z axis at (x, y):
    # t = oz, u = x, v = y.  dt/dv0_z: moving the whole plane up by dz at a
    # weight (1-u-v) lowers t by (1-u-v) dz; du/dv1_x = -u (shrinking the
    # first edge scales u = x/len) and du/do_x = 1.
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float64)
    f = np.array([[0, 1, 2]], np.uint32)
    x, y, oz = 0.25, 0.125, 2.0
    rays = np.array([[x, y, oz, 0, 0, 0, -1, np.inf]], np.float32)
    prims = np.array([0], np.uint32)
    gv, gr = oracle_lib.hit_grad64(v, f, rays, prims, np.array([[1.0, 0.0, 0.0]]))
    w0 = 1 - x - y
    assert np.allclose(gv[:, 2], [-w0, -x, -y])         # dt/dv_k,z
    assert np.allclose(gv[:, :2], 0)
    assert np.allclose(gr[0, :3], [0, 0, 1.0])          # t = oz for d = -z: dt/do_z = 1
    gv, gr = oracle_lib.hit_grad64(v, f, rays, prims, np.array([[0.0, 1.0, 0.0]]))
    assert np.isclose(gv[1, 0], -x) and np.isclose(gr[0, 0], 1.0)
