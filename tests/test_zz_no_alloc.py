"""rt_trace_closest_noalloc (the allocation-free variant of rt_trace_closest,
whose workspace is the library's fixed device scratch) against
rt_trace_closest with a caller workspace, through the C ABI: bit-identical
hits and counters on two calls in a row, the second with a smaller input,
so that the scratch still holds the first call's queue heads and spilled
stack entries when the second starts.

Call 1: alpha-masked billboards, 200k triangles, 1920x1080 rays, counting,
the default (persistent, ray-queue) launch shape.  Call 2: the tiny scene,
1,024 triangles and 64x64 rays, accept-all, no counters.  A third call
repeats the first on a deep BVH (a stack that spills past the on-chip ring
into the scratch)."""
import numpy as np
import pytest

from paper_1912_12786_amd import workloads as W

pytestmark = pytest.mark.gpu


def _both(rtx, torch, scene, rays, kind, count, alpha_min=128, flags=0):
    n = rays.shape[0]
    sc = scene.view
    params = rtx._params(scene, kind, alpha_min, 8)
    k = rtx.KINDS[kind]
    flags |= rtx.RT_FLAG_COUNT if count else 0
    stream = torch.cuda.current_stream().cuda_stream
    h_ref = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    c_ref = torch.empty((n, 4), dtype=torch.int32, device="cuda") if count else None
    wb = rtx.rt_trace_workspace_bytes(sc, n, flags)
    ws = torch.empty(max(wb, 16), dtype=torch.uint8, device="cuda")
    rtx.rt_trace_closest(sc, rays.data_ptr(), n, k, params, flags, h_ref.data_ptr(),
                         c_ref.data_ptr() if count else None, ws.data_ptr(), wb, stream)
    h = torch.full((n, 4), 7.0, dtype=torch.float32, device="cuda")
    c = torch.full((n, 4), 7, dtype=torch.int32, device="cuda") if count else None
    rtx.rt_trace_closest_noalloc(sc, rays.data_ptr(), n, k, params, flags, h.data_ptr(),
                                 c.data_ptr() if count else None, stream)
    torch.cuda.synchronize()
    assert torch.equal(h.view(torch.int32), h_ref.view(torch.int32)), "hits differ"
    if count:
        assert torch.equal(c, c_ref), "counters differ"
    return h.cpu().numpy(), wb


def test_noalloc_matches_workspace_entry_point():
    import torch
    from paper_1912_12786_amd import rtx
    rtx.load_library()
    print("[gpu-case] noalloc call 1: billboards 200k tris, 1920x1080, alpha, counters",
          flush=True)
    wl = W.billboards()
    scene = rtx.upload_scene(wl.vertices, wl.geom_ids, wl.texcoords, wl.textures, max_leaf=2)
    assert scene.info.max_depth <= 22
    rays = torch.from_numpy(wl.rays).cuda()
    h1, wb1 = _both(rtx, torch, scene, rays, "alpha", True)
    assert wb1 > 1024, "the first call should use spill space as well as the queue heads"
    assert wb1 <= rtx.RT_NOALLOC_SCRATCH_BYTES
    assert (h1[:, 1].view(np.uint32) != rtx.RT_MISS).sum() > 100_000

    print("[gpu-case] noalloc call 2: tiny 1,024 tris, 64x64, default, no counters", flush=True)
    tw = W.tiny()
    tscene = rtx.upload_scene(tw.vertices)
    trays = torch.from_numpy(tw.rays).cuda()
    h2, _ = _both(rtx, torch, tscene, trays, "default", False)
    assert (h2[:, 1].view(np.uint32) != rtx.RT_MISS).sum() > 100

    print("[gpu-case] noalloc call 3: deep BVH (stacked coplanar-offset slabs), spill", flush=True)
    # 4,096 thin triangles stacked along z: a BVH whose depth exceeds the
    # 7-entry on-chip ring, traversed by rays along z (every level pushes)
    n = 4096
    rng = np.random.default_rng(3)
    z = np.sort(rng.uniform(0, 10, n)).astype(np.float32)
    v = np.zeros((n, 3, 3), np.float32)
    v[:, 0] = np.stack([np.zeros(n), np.zeros(n), z], 1)
    v[:, 1] = np.stack([np.ones(n), np.zeros(n), z], 1)
    v[:, 2] = np.stack([np.zeros(n), np.ones(n), z], 1)
    dscene = rtx.upload_scene(v, max_leaf=1)
    assert 7 < dscene.info.max_depth <= 22, dscene.info.max_depth
    m = 20_000
    r = np.zeros((m, 8), np.float32)
    r[:, 0:2] = rng.uniform(0.01, 0.49, size=(m, 2))
    r[:, 2] = 11.0
    r[:, 6] = -1.0
    r[:, 7] = np.inf
    h3, wb3 = _both(rtx, torch, dscene, torch.from_numpy(r).cuda(), "default", True)
    assert wb3 > 1024
    assert np.all(h3[:, 1].view(np.uint32) != rtx.RT_MISS)
