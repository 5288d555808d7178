"""Pins of the multi-hit oracles: the hand-derived layered-quads fixture,
k = 1 reducing to the closest-hit query, and oracle B against oracle A."""
import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from tests.golden.load import load, uniform_alpha_textures
from tests.test_oracle_pins import _random_scene, _scene_params

MISS = 0xFFFFFFFF


def test_golden_layers(oracle_lib):
    fx = load("layers.json")
    bvh = oracle_lib.build_bvh(fx["vertices"])
    for case in fx["cases"]:
        k = case["k"]
        tex = uniform_alpha_textures(case["alpha"], fx["texture_size"])
        kw = dict(geom_ids=fx["geom_ids"], texcoords=fx["texcoords"], textures=tex, alpha_min=128)
        A = oracle_lib.brute_multi(fx["vertices"], fx["rays"], k, "alpha", **kw)
        B = oracle_lib.traverse(fx["vertices"], bvh, fx["rays"], "alpha", multi_k=k, **kw)
        n = len(case["prims"])
        for R in (A, B):
            assert R["n_hits"][0] == n
            assert R["prim"][0, :n].tolist() == case["prims"]
            assert R["t"][0, :n].tolist() == case["t"]
            assert np.all(R["prim"][0, n:] == MISS) and np.all(np.isinf(R["t"][0, n:]))
            assert np.all(R["u"][0, :n] == 0.625) and np.all(R["v"][0, :n] == 0.0625)


def test_multi_k1_is_closest_hit(oracle_lib):
    rng = np.random.default_rng(12)
    verts, rays = _random_scene(rng, 60, 300)
    for kind in ("default", "alpha", "procedural"):
        kw = _scene_params(rng, kind, verts.shape[0])
        bvh = oracle_lib.build_bvh(verts)
        c = oracle_lib.traverse(verts, bvh, rays, kind, **kw)
        m = oracle_lib.traverse(verts, bvh, rays, kind, multi_k=1, **kw)
        assert np.array_equal(m["prim"][:, 0], c["prim"])
        for key in ("t", "u", "v"):
            assert np.array_equal(m[key][:, 0].view(np.uint32), c[key].view(np.uint32))
        assert np.array_equal(m["counters"], c["counters"])
        assert np.array_equal(m["n_hits"], (c["prim"] != MISS).astype(np.uint32))
        a = oracle_lib.brute(verts, rays, kind, **kw)
        am = oracle_lib.brute_multi(verts, rays, 1, kind, **kw)
        ok = (a["flags"] == 0) & (am["flags"] == 0)
        assert np.array_equal(am["prim"][ok, 0], a["prim"][ok])


@settings(max_examples=25, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2**31 - 1), n_tris=st.integers(1, 64), k=st.integers(1, 8),
       kind=st.sampled_from(["default", "alpha", "procedural"]))
def test_multi_oracle_b_matches_a(oracle_lib, seed, n_tris, k, kind):
    rng = np.random.default_rng(seed)
    verts, rays = _random_scene(rng, n_tris, 128)
    kw = _scene_params(rng, kind, n_tris)
    bvh = oracle_lib.build_bvh(verts)
    A = oracle_lib.brute_multi(verts, rays, k, kind, **kw)
    B = oracle_lib.traverse(verts, bvh, rays, kind, multi_k=k, **kw)
    ok = A["flags"] == 0
    assert np.array_equal(A["n_hits"][ok], B["n_hits"][ok])
    assert np.array_equal(A["prim"][ok], B["prim"][ok])
    # t within max(1e-5 |t|, B_t) (plus an absolute floor for hits very close
    # to the origin), B_t being the a-priori float32 error bound of that
    # ray-triangle pair, as for the closest hit
    for i, j in zip(*np.nonzero(ok[:, None] & (A["prim"] != MISS))):
        p = int(A["prim"][i, j])
        one = oracle_lib.brute(verts[p:p + 1], rays[i:i + 1], "default")
        tol = max(1e-5 * abs(A["t"][i, j]), one["bound_t"][0]) + 1e-6
        assert abs(A["t"][i, j] - B["t"][i, j]) <= tol, (i, j, A["t"][i, j], B["t"][i, j], tol)
    # kept distances are sorted and the list is padded with misses
    for R in (A, B):
        t = R["t"]
        assert np.all(t[:, :-1] <= t[:, 1:])
        assert np.all((R["prim"] == MISS) == (np.arange(k)[None, :] >= R["n_hits"][:, None]))
