"""The runtime-dispatched intersectors (an inlined run-time switch, and an
indirect call through a table of filter functions) must give bit-identical
results to the compile-time intersectors, and all three equal oracle B."""
import numpy as np
import pytest

from paper_1912_12786_amd import workloads as W

pytestmark = pytest.mark.gpu


def same_bits(a, b):
    import torch
    return a.shape == b.shape and torch.equal(a.view(torch.int32), b.view(torch.int32))


def trace_flags(torch, rtx, scene, rays, kind, flags, **kw):
    n = rays.shape[0]
    out = torch.empty((n, 4), dtype=torch.float32, device="cuda")
    params = rtx._params(scene, kind, kw.get("alpha_min", 128), kw.get("checker_n", 8))
    sc = scene.view
    ws = rtx.Workspace("cuda")
    wptr, wb = ws.get(rtx.rt_trace_workspace_bytes(sc, n, flags))
    rtx.rt_trace_closest(sc, rays.data_ptr(), n, rtx.KINDS[kind], params, flags, out.data_ptr(),
                         None, wptr, wb, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("workload", ["tiny", "billboards"])
@pytest.mark.parametrize("kind", ["default", "alpha", "procedural"])
def test_runtime_dispatch_is_bit_identical(oracle_lib, workload, kind):
    import torch
    from paper_1912_12786_amd import rtx
    print(f"[gpu-case] runtime dispatch {workload} {kind}", flush=True)
    if workload == "tiny":
        wl = W.tiny()
        rng = np.random.default_rng(3)
        tex = W.alpha_textures(4, 64, 3)
        geom = rng.integers(0, 4, size=wl.n_tris).astype(np.uint32)
        tc = rng.uniform(0, 1, size=(wl.n_tris, 3, 2)).astype(np.float32)
        scene = rtx.upload_scene(wl.vertices, geom, tc, tex)
    else:
        wl = W.billboards()
        scene = rtx.upload_scene(wl.vertices, wl.geom_ids, wl.texcoords, wl.textures)
    rays = torch.from_numpy(wl.rays).cuda()
    ref = rtx.trace(scene, rays, kind, alpha_min=128, checker_n=8)
    for flags in (rtx.RT_FLAG_RUNTIME_SWITCH, rtx.RT_FLAG_RUNTIME_CALL):
        got = trace_flags(torch, rtx, scene, rays, kind, flags)
        assert same_bits(got, ref), flags
    # and all three against oracle B (the same BVH, leaves of at most 4)
    okw = {}
    if kind == "alpha":
        okw = dict(geom_ids=geom, texcoords=tc, textures=tex, alpha_min=128) if workload == "tiny" \
            else dict(geom_ids=wl.geom_ids, texcoords=wl.texcoords, textures=wl.textures,
                      alpha_min=128)
    elif kind == "procedural":
        okw = dict(checker_n=8)
    B = oracle_lib.traverse(wl.vertices, oracle_lib.build_bvh(wl.vertices), wl.rays, kind,
                            count=False, **okw)
    from tests import parity as P
    P.assert_exact_vs_b(P.hits_to_numpy(ref), B, f"dispatch {workload} {kind}")
