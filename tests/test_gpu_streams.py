"""Launch shape and stream are per call: two side streams running the same
trace concurrently with different launch shapes, each allocating its outputs
and a temporary workspace through ``stream=``, give the bits of a plain call
on torch's current stream (alpha mask, closest hit with counters, billboards
200k triangles at 1920x1080)."""
import pytest

from paper_1912_12786_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_two_streams_two_shapes(tmp_path):
    import torch
    from paper_1912_12786_amd import rtx
    rtx.load_library()
    wl = W.billboards()
    scene = rtx.upload_scene(wl.vertices, wl.geom_ids, wl.texcoords, wl.textures, max_leaf=2)
    rays = torch.from_numpy(wl.rays).cuda()
    shapes = rtx.rt_launch_shapes()
    print(f"[gpu-case] two side streams, shapes {shapes[0]} and {shapes[3]}", flush=True)
    ref_h, ref_c = rtx.trace(scene, rays, "alpha", alpha_min=128, count=True)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    outs = []
    for _ in range(3):   # repeated, so freed temporaries are reused while others run
        a = rtx.trace(scene, rays, "alpha", alpha_min=128, count=True, stream=s1.cuda_stream,
                      shape=shapes[0])
        b = rtx.trace(scene, rays, "alpha", alpha_min=128, count=True, stream=s2.cuda_stream,
                      shape=shapes[3])
        outs.append((a, b))
    torch.cuda.synchronize()
    for a, b in outs:
        for h, c in (a, b):
            assert torch.equal(h.view(torch.int32), ref_h.view(torch.int32))
            assert torch.equal(c, ref_c)
