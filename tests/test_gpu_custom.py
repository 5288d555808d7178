"""A user-defined intersector (tests/custom/prim_mask.hip: keep a hit iff
mask[prim_id] != 0) compiled against the traversal template.

Its results equal, bit for bit and with all four counters, the built-in alpha
intersector on textures that encode the same decision (texture 0 fully
transparent, texture 1 fully opaque, geom_id = mask), which oracle B checks
exactly; and the closest kept hit is the float64 closest hit of the sub-scene
of kept triangles (oracle A on that sub-scene, outside its exception set)."""
import numpy as np
import pytest

from paper_1912_12786_amd import workloads as W
from tests import parity as P

pytestmark = pytest.mark.gpu
MISS = 0xFFFFFFFF


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_1912_12786_amd import rtx
    from tests.custom import binding
    rtx.load_library()
    binding.load()
    return torch, rtx, binding


def mask_textures():
    # texture 0: alpha 0 (reject); texture 1: alpha 255 (accept); 1x1 texels
    return np.array([[[0x00000000]], [[0xFF000000]]], np.uint32)


@pytest.mark.parametrize("workload", ["tiny", "billboards"])
def test_custom_mask_intersector(env, oracle_lib, workload):
    torch, rtx, binding = env
    wl = W.tiny() if workload == "tiny" else W.billboards()
    rng = np.random.default_rng(31)
    mask = (rng.uniform(size=wl.n_tris) < 0.6).astype(np.uint8)
    announce(f"custom per-primitive mask intersector, {wl.name}, {int(mask.sum())} kept")
    scene = rtx.upload_scene(wl.vertices)
    rays = torch.from_numpy(wl.rays).cuda()
    m = torch.from_numpy(mask).cuda()
    hits, cnt = binding.trace(scene, rays, m, count=True)
    plain = binding.trace(scene, rays, m)
    # the built-in alpha intersector making the same decision
    geom = mask.astype(np.uint32)
    tc = np.zeros((wl.n_tris, 3, 2), np.float32)
    tex = mask_textures()
    ascene = rtx.upload_scene(wl.vertices, geom, tc, tex)
    ah, ac = rtx.trace(ascene, rays, "alpha", alpha_min=128, count=True)
    torch.cuda.synchronize()
    assert torch.equal(hits.view(torch.int32), ah.view(torch.int32))
    assert torch.equal(cnt, ac)
    assert torch.equal(plain.view(torch.int32), hits.view(torch.int32))
    # oracle B with the same encoding, bit for bit
    bvh = oracle_lib.build_bvh(wl.vertices)
    idx = np.arange(wl.n_rays) if workload == "tiny" else np.arange(0, wl.n_rays, 7)
    B = oracle_lib.traverse(wl.vertices, bvh, wl.rays[idx], "alpha", geom_ids=geom, texcoords=tc,
                            textures=tex, alpha_min=128)
    g = P.hits_to_numpy(hits)
    P.assert_exact_vs_b({k: v[idx] for k, v in g.items()}, B, "custom mask")
    assert np.array_equal(cnt.cpu().numpy().view(np.uint32)[idx], B["counters"])
    # the definition: closest hit of the kept sub-scene
    keep = np.nonzero(mask)[0]
    sub = W.subsample_indices(wl.n_rays, None, None, seed=3, n_random=2048)
    A = oracle_lib.brute(wl.vertices[keep], wl.rays, "default", ray_index=sub)
    ok = A["flags"] == 0
    gp = g["prim"][sub]
    mapped = np.where(A["prim"] == MISS, MISS, keep[np.minimum(A["prim"], len(keep) - 1)])
    assert ok.mean() > 0.9
    assert np.array_equal(gp[ok], mapped[ok].astype(np.uint32))
    assert (gp != MISS).mean() > 0.1
