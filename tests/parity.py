"""Comparison helpers for the GPU parity tests.

Parity bar (stated here and applied in every GPU test):
* against oracle B (float32 traversal of the same BVH, same operation
  sequence): bit-exact t, u, v, prim_id, occluders and all four counters,
  for every ray;
* against oracle A (float64 brute force, the plain definition): prim_id
  exact for every ray outside the exception set E (near ties, near-edge
  candidates, near filter decisions); t within max(1e-5 |t|, B_t) and u, v
  within max(1e-5, B_uv), where B_t and B_uv are oracle A's a-priori
  float32 forward-error bounds for that hit.
"""
import numpy as np

MISS = 0xFFFFFFFF


def hits_to_numpy(hits):
    h = hits.detach().cpu().numpy()
    return {"t": h[:, 0].copy(), "prim": h[:, 1].view(np.uint32).copy(),
            "u": h[:, 2].copy(), "v": h[:, 3].copy()}


def bits(x):
    return np.ascontiguousarray(x, np.float32).view(np.uint32)


def assert_exact_vs_b(gpu, B, what=""):
    """Closest-hit records bit-identical to oracle B."""
    n = len(B["prim"])
    bad = np.nonzero(gpu["prim"] != B["prim"])[0]
    assert bad.size == 0, f"{what}: prim differs on {bad.size}/{n} rays, first {bad[:5]}"
    for k in ("t", "u", "v"):
        bad = np.nonzero(bits(gpu[k]) != bits(B[k]))[0]
        assert bad.size == 0, (f"{what}: {k} differs on {bad.size}/{n} rays, first {bad[:5]}: "
                               f"gpu {gpu[k][bad[:3]]} oracle {B[k][bad[:3]]}")


def assert_counters_vs_b(cnt, B, what=""):
    c = cnt.detach().cpu().numpy().view(np.uint32)
    bad = np.nonzero(np.any(c != B["counters"], axis=1))[0]
    assert bad.size == 0, (f"{what}: counters differ on {bad.size} rays, first {bad[:5]}: "
                           f"gpu {c[bad[:3]].tolist()} oracle {B['counters'][bad[:3]].tolist()}")


def compare_vs_a(gpu, A, idx, what="", any_hit=False):
    """prim exact outside E, t/u/v within tolerance.  Returns a summary."""
    ok = A["flags"] == 0
    gp = gpu["prim"][idx]
    if any_hit:
        bad = np.nonzero(((gp == MISS) != (A["prim"] == MISS)) & ok)[0]
        assert bad.size == 0, f"{what}: occlusion differs outside E on {bad.size} rays"
        return {"checked": int(ok.sum()), "excluded": int((~ok).sum())}
    bad = np.nonzero((gp != A["prim"]) & ok)[0]
    assert bad.size == 0, (f"{what}: prim differs from the float64 definition outside E on "
                           f"{bad.size}/{ok.sum()} rays, first ray ids {np.asarray(idx)[bad[:5]]}")
    hit = ok & (A["prim"] != MISS)
    dt = np.abs(gpu["t"][idx][hit].astype(np.float64) - A["t"][hit])
    du = np.abs(gpu["u"][idx][hit].astype(np.float64) - A["u"][hit])
    dv = np.abs(gpu["v"][idx][hit].astype(np.float64) - A["v"][hit])
    tol_t = np.maximum(1e-5 * np.abs(A["t"][hit]), A["bound_t"][hit])
    tol_uv = np.maximum(1e-5, A["bound_uv"][hit])
    assert np.all(dt <= tol_t), f"{what}: t outside tolerance on {(dt > tol_t).sum()} rays"
    assert np.all(du <= tol_uv), f"{what}: u outside tolerance on {(du > tol_uv).sum()} rays"
    assert np.all(dv <= tol_uv), f"{what}: v outside tolerance on {(dv > tol_uv).sum()} rays"
    rel_t = dt / np.maximum(np.abs(A["t"][hit]), 1e-30)
    return {"checked": int(ok.sum()), "excluded": int((~ok).sum()),
            "max_rel_t": float(rel_t.max()) if rel_t.size else 0.0,
            "max_uv": float(max(du.max(), dv.max())) if du.size else 0.0,
            "n_uv_over_1e-5": int(((du > 1e-5) | (dv > 1e-5)).sum())}


def occluders_to_numpy(occ):
    return occ.detach().cpu().numpy().view(np.uint32).copy()
