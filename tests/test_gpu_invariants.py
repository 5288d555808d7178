"""Per-ray invariants of the GPU results that need no oracle traversal, at the
benchmark's size (billboards, 200k triangles, 1920x1080, alpha >= 128):

* certificate: every reported hit is a geometric hit of its triangle (the
  point o + t d and the barycentric point agree to 1e-5 max(1, |o|, t) in
  float64) and its alpha decision, re-evaluated on the host, accepts it;
* filtering never brings a hit nearer: t(alpha) >= t(accept-all) per ray;
* ray order: the same rays in 8x8 tiles or Z-order give the same per-ray
  hits and counters;
* repeated launches give identical hits and counters;
* every compiled launch shape gives the same bits (closest with counters,
  4 nearest hits)."""
import numpy as np
import pytest

from paper_1912_12786_amd import workloads as W
from tests import parity as P

pytestmark = pytest.mark.gpu
MISS = 0xFFFFFFFF


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available()
    from paper_1912_12786_amd import rtx
    rtx.load_library()
    wl = W.billboards()
    scene = rtx.upload_scene(wl.vertices, wl.geom_ids, wl.texcoords, wl.textures, max_leaf=2)
    return torch, rtx, wl, scene


def test_hit_certificates(setup):
    torch, rtx, wl, scene = setup
    announce("billboards alpha: per-hit certificates")
    rays = torch.from_numpy(wl.rays).cuda()
    hits = rtx.trace(scene, rays, "alpha", alpha_min=128)
    dflt = rtx.trace(scene, rays, "default")
    torch.cuda.synchronize()
    g = P.hits_to_numpy(hits)
    d = P.hits_to_numpy(dflt)
    hit = np.nonzero(g["prim"] != MISS)[0]
    assert hit.size > 0.2 * wl.n_rays
    prim = g["prim"][hit].astype(np.int64)
    o = wl.rays[hit, :3].astype(np.float64)
    dirs = wl.rays[hit, 4:7].astype(np.float64)
    t = g["t"][hit].astype(np.float64)
    u = g["u"][hit].astype(np.float64)
    v = g["v"][hit].astype(np.float64)
    tri = wl.vertices[prim].astype(np.float64)
    p_ray = o + t[:, None] * dirs
    p_bary = (1 - u - v)[:, None] * tri[:, 0] + u[:, None] * tri[:, 1] + v[:, None] * tri[:, 2]
    scale = np.maximum(np.maximum(1.0, np.linalg.norm(o, axis=1)), t)
    assert np.all(np.linalg.norm(p_ray - p_bary, axis=1) <= 1e-5 * scale)
    assert np.all((u >= 0) & (v >= 0) & (u + v <= 1 + 1e-6))
    # the alpha decision, re-evaluated in float64 away from texel edges
    tc = wl.texcoords[prim].astype(np.float64)
    s = (1 - u - v) * tc[:, 0, 0] + u * tc[:, 1, 0] + v * tc[:, 2, 0]
    tt = (1 - u - v) * tc[:, 0, 1] + u * tc[:, 1, 1] + v * tc[:, 2, 1]
    h, w = wl.textures.shape[1:]
    xs, ys = s * w, tt * h
    clear = (np.abs(xs - np.round(xs)) > 1e-3) & (np.abs(ys - np.round(ys)) > 1e-3)
    x = np.clip(np.floor(xs), 0, w - 1).astype(np.int64)
    y = np.clip(np.floor(ys), 0, h - 1).astype(np.int64)
    a8 = wl.textures[wl.geom_ids[prim], y, x] >> 24
    assert clear.mean() > 0.99
    assert np.all(a8[clear] >= 128)
    # filtering never brings a hit nearer than the accept-all closest hit
    assert np.all(d["prim"][hit] != MISS)
    assert np.all(g["t"][hit] >= d["t"][hit])


@pytest.mark.parametrize("order", ["tiled", "morton"])
def test_ray_order_invariance(setup, order):
    import bench
    torch, rtx, wl, scene = setup
    announce(f"billboards alpha: scanline vs {order} ray order")
    perm = bench.tile_order(wl, morton=(order == "morton"))
    h0, c0 = rtx.trace(scene, torch.from_numpy(wl.rays).cuda(), "alpha", alpha_min=128, count=True)
    h1, c1 = rtx.trace(scene, torch.from_numpy(np.ascontiguousarray(wl.rays[perm])).cuda(), "alpha",
                       alpha_min=128, count=True)
    torch.cuda.synchronize()
    p = torch.from_numpy(perm).cuda()
    assert torch.equal(h0[p].view(torch.int32), h1.view(torch.int32))
    assert torch.equal(c0[p], c1)


def test_repeated_launches_identical(setup):
    torch, rtx, wl, scene = setup
    announce("billboards alpha: 10 repeated launches")
    rays = torch.from_numpy(wl.rays).cuda()
    ref_h, ref_c = rtx.trace(scene, rays, "alpha", alpha_min=128, count=True)
    for _ in range(10):
        h, c = rtx.trace(scene, rays, "alpha", alpha_min=128, count=True)
        torch.cuda.synchronize()
        assert torch.equal(h.view(torch.int32), ref_h.view(torch.int32)) and torch.equal(c, ref_c)


def test_all_launch_shapes_identical_full_size(setup):
    """Every compiled launch shape, in one process and in turn, gives the
    same bits for the closest hit with its counters and for the 4 nearest
    hits: the per-ray visit order does not depend on the shape, the grid or
    how many waves are resident."""
    torch, rtx, wl, scene = setup
    rays = torch.from_numpy(wl.rays).cuda()
    shapes = rtx.rt_launch_shapes()
    ref = None
    for shape in shapes:
        announce(f"billboards alpha closest+count and multi k=4, shape={shape}")
        h, c = rtx.trace(scene, rays, "alpha", alpha_min=128, count=True, shape=shape)
        m, n = rtx.trace(scene, rays, "alpha", query="multi", k=4, alpha_min=128, shape=shape)
        torch.cuda.synchronize()
        got = (h.view(torch.int32), c, m.view(torch.int32), n)
        if ref is None:
            ref = got
        else:
            assert all(torch.equal(x, y) for x, y in zip(got, ref)), shape
