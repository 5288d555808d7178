"""The tiled schedule (RT_FLAG_TILE_WIDTH: lanes take the rays of an image in
8 x 8 pixel tiles) changes only which lanes trace which rays: every result
and counter, at its ray's index, equals the call in index order, for every
query, node layout and entry point, including ray counts that end inside a
row of tiles; a sentinel-filled output shows that every ray is traced once."""
import numpy as np
import pytest

from paper_1912_12786_amd import workloads as W
from tests import parity as P

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_1912_12786_amd import rtx
    rtx.load_library()
    return torch, rtx


def same_bits(a, b):
    import torch
    return a.shape == b.shape and torch.equal(a.view(torch.int32), b.view(torch.int32))


@pytest.fixture(scope="module")
def billboards(env):
    torch, rtx = env
    wl = W.billboards()
    scenes = {layout: rtx.upload_scene(wl.vertices, wl.geom_ids, wl.texcoords, wl.textures,
                                       max_leaf=2, layout=layout)
              for layout in ("f32", "q8", "f32p", "wide4")}
    return wl, scenes, torch.from_numpy(wl.rays).cuda()


@pytest.mark.parametrize("layout", ["f32", "q8", "f32p", "wide4"])
def test_tiled_schedule_matches_index_order(env, billboards, layout):
    torch, rtx = env
    wl, scenes, rays = billboards
    sc = scenes[layout]
    for query in ("closest", "any", "multi"):
        announce(f"billboards alpha {layout} {query}: tiles of the 1920-wide image vs index order")
        ref, rc = rtx.trace(sc, rays, "alpha", query=query, k=2, count=True, alpha_min=128)
        if query == "closest":
            out = torch.full((wl.n_rays, 4), 7.0, device="cuda")
            got, gc = rtx.trace(sc, rays, "alpha", query=query, count=True, alpha_min=128,
                                out=out, image_width=1920)
        else:
            got, gc = rtx.trace(sc, rays, "alpha", query=query, k=2, count=True, alpha_min=128,
                                image_width=1920)
        torch.cuda.synchronize()
        if query == "multi":
            assert same_bits(got[0], ref[0]) and same_bits(got[1], ref[1])
        else:
            assert same_bits(got, ref)
        assert same_bits(gc, rc)


@pytest.mark.parametrize("n,width", [(2_073_600 - 1234, 1920), (2_073_600, 1912), (200, 8),
                                     (100, 24), (64 * 64, 64)])
def test_tiled_schedule_partial_rows(env, oracle_lib, billboards, n, width):
    """Ray counts that end inside a row of tiles, widths that do not divide
    the count, and fewer rays than one row of tiles: the tiled part is the
    whole rows of tiles, the rest keeps index order; the result equals index
    order and oracle B."""
    torch, rtx = env
    wl, scenes, rays = billboards
    announce(f"tiled schedule n={n} width={width}")
    r = rays[:n].contiguous()
    out = torch.full((n, 4), 7.0, device="cuda")
    got, gc = rtx.trace(scenes["f32"], r, "alpha", count=True, alpha_min=128, out=out,
                        image_width=width)
    ref, rc = rtx.trace(scenes["f32"], r, "alpha", count=True, alpha_min=128)
    torch.cuda.synchronize()
    assert same_bits(got, ref) and same_bits(gc, rc)
    if n <= 5000:
        okw = dict(geom_ids=wl.geom_ids, texcoords=wl.texcoords, textures=wl.textures,
                   alpha_min=128)
        B = oracle_lib.traverse(wl.vertices, oracle_lib.build_bvh(wl.vertices, max_leaf=2),
                                wl.rays[:n], "alpha", **okw)
        P.assert_exact_vs_b(P.hits_to_numpy(got), B, f"tiled n={n}")
        P.assert_counters_vs_b(gc, B, f"tiled n={n}")


def test_tiled_schedule_noalloc_and_spheres(env):
    """The allocation-free entry point with the tile flag, and the spheres'
    primary rays tiled while their bounce rays keep index order."""
    torch, rtx = env
    wl = W.spheres()
    sc = rtx.upload_scene(wl.vertices, layout="q8", max_leaf=2)
    rays = torch.from_numpy(wl.rays).cuda()
    announce("spheres procedural, tiled primary rays")
    ref = rtx.trace(sc, rays, "procedural", checker_n=8)
    got = rtx.trace(sc, rays, "procedural", checker_n=8, image_width=1920)
    torch.cuda.synchronize()
    assert same_bits(got, ref)
    tw = W.tiny()
    tsc = rtx.upload_scene(tw.vertices)
    trays = torch.from_numpy(tw.rays).cuda()
    announce("noalloc tiny, tiled 64-wide image")
    h = torch.full((tw.n_rays, 4), 7.0, device="cuda")
    rtx.rt_trace_closest_noalloc(tsc.view, trays.data_ptr(), tw.n_rays, 0, None,
                                 rtx.tile_flag(64), h.data_ptr(), None,
                                 torch.cuda.current_stream().cuda_stream)
    ref = rtx.trace(tsc, trays)
    torch.cuda.synchronize()
    assert same_bits(h, ref)


@pytest.mark.parametrize("layout", ["f32", "q8", "f32p", "wide4"])
def test_longest_first_matches_index_order(env, billboards, layout):
    """Longest-path-first chunk order (with and without tiles) equals index
    order for every query and node layout."""
    torch, rtx = env
    wl, scenes, rays = billboards
    sc = scenes[layout]
    for query in ("closest", "any", "multi"):
        ref, rc = rtx.trace(sc, rays, "alpha", query=query, k=2, count=True, alpha_min=128)
        for width in (None, 1920):
            announce(f"billboards alpha {layout} {query} longest-first tiles={width}")
            if query == "closest":
                out = torch.full((wl.n_rays, 4), 7.0, device="cuda")
                got, gc = rtx.trace(sc, rays, "alpha", count=True, alpha_min=128, out=out,
                                    image_width=width, longest_first=True)
            else:
                got, gc = rtx.trace(sc, rays, "alpha", query=query, k=2, count=True,
                                    alpha_min=128, image_width=width, longest_first=True)
            torch.cuda.synchronize()
            if query == "multi":
                assert same_bits(got[0], ref[0]) and same_bits(got[1], ref[1])
            else:
                assert same_bits(got, ref)
            assert same_bits(gc, rc)


def test_longest_first_every_shape_and_size(env, oracle_lib, billboards):
    """Every compiled launch shape (static and persistent grids, chunks of 32,
    64 and 128), ray counts that end inside a chunk, one ray, and the
    allocation-free entry point; sentinel-filled outputs."""
    torch, rtx = env
    wl, scenes, rays = billboards
    sc = scenes["f32"]
    for shape in rtx.rt_launch_shapes():
        for n in (1, 63, 100_001, wl.n_rays):
            announce(f"longest-first shape={tuple(shape)} n={n}")
            r = rays[:n].contiguous()
            out = torch.full((n, 4), 7.0, device="cuda")
            got = rtx.trace(sc, r, "alpha", alpha_min=128, out=out, shape=tuple(shape),
                            longest_first=True, image_width=1920 if n == wl.n_rays else None)
            ref = rtx.trace(sc, r, "alpha", alpha_min=128, shape=tuple(shape))
            torch.cuda.synchronize()
            assert same_bits(got, ref), (tuple(shape), n)
    announce("longest-first through rt_trace_closest_noalloc")
    h = torch.full((wl.n_rays, 4), 7.0, device="cuda")
    flags = rtx.RT_FLAG_LONGEST_FIRST | rtx.tile_flag(1920)
    rtx.rt_trace_closest_noalloc(sc.view, rays.data_ptr(), wl.n_rays, rtx.KINDS["alpha"],
                                 rtx._params(sc, "alpha", 128, 8), flags, h.data_ptr(), None,
                                 torch.cuda.current_stream().cuda_stream)
    ref = rtx.trace(sc, rays, "alpha", alpha_min=128)
    torch.cuda.synchronize()
    assert same_bits(h, ref)


def test_longest_first_spheres_and_empty(env):
    torch, rtx = env
    wl = W.spheres()
    sc = rtx.upload_scene(wl.vertices, layout="q8", max_leaf=2)
    rays = torch.from_numpy(wl.rays).cuda()
    announce("spheres procedural longest-first with counters")
    ref, rc = rtx.trace(sc, rays, "procedural", checker_n=8, count=True)
    got, gc = rtx.trace(sc, rays, "procedural", checker_n=8, count=True, longest_first=True)
    torch.cuda.synchronize()
    assert same_bits(got, ref) and same_bits(gc, rc)
    announce("longest-first on an empty scene")
    empty = rtx.upload_scene(np.zeros((0, 3, 3), np.float32))
    h = rtx.trace(empty, rays[:1000].contiguous(), longest_first=True)
    torch.cuda.synchronize()
    assert np.all(P.hits_to_numpy(h)["prim"] == 0xFFFFFFFF)


@pytest.mark.parametrize("waves", [1, 3, 5, 8, 15])
def test_waves_per_simd_matches_default(env, billboards, waves):
    """Capping the persistent grid (RT_FLAG_WAVES_PER_SIMD, which sets the
    rays each lane traces) changes no result or counter: closest, any and
    multi-hit with counters, tiled and longest-first, every queue shape, into
    sentinel-filled outputs, against the default grid (7)."""
    torch, rtx = env
    wl, scenes, rays = billboards
    sc = scenes["f32"]
    for query in ("closest", "any", "multi"):
        announce(f"billboards alpha {query}: {waves} waves per SIMD vs the default grid")
        ref, rc = rtx.trace(sc, rays, "alpha", query=query, k=2, count=True, alpha_min=128)
        if query == "closest":
            out = torch.full((wl.n_rays, 4), 7.0, device="cuda")
            got, gc = rtx.trace(sc, rays, "alpha", count=True, alpha_min=128, out=out,
                                image_width=1920, longest_first=True, waves_per_simd=waves)
        else:
            got, gc = rtx.trace(sc, rays, "alpha", query=query, k=2, count=True, alpha_min=128,
                                waves_per_simd=waves)
        torch.cuda.synchronize()
        if query == "multi":
            assert same_bits(got[0], ref[0]) and same_bits(got[1], ref[1])
        else:
            assert same_bits(got, ref)
        assert same_bits(gc, rc)
    r = rays[:300_001].contiguous()
    ref = rtx.trace(sc, r, "default")
    for shape in rtx.rt_launch_shapes():
        if not shape[3]:
            continue
        announce(f"billboards default, 300001 rays, shape {tuple(shape)}, {waves} waves per SIMD")
        got = rtx.trace(sc, r, "default", shape=tuple(shape), waves_per_simd=waves)
        torch.cuda.synchronize()
        assert same_bits(got, ref)


def test_waves_per_simd_batch(env):
    """A batched launch with its grid capped at 1 and at 4 waves per SIMD
    equals the default grid, hits and counters."""
    torch, rtx = env
    scenes = [W.tiny(), W.tiny()]
    sc_list = [rtx.upload_scene(s.vertices) for s in scenes]
    rays = torch.from_numpy(np.concatenate([scenes[0].rays, scenes[1].rays[:777]])).cuda()
    batch = rtx.Batch(sc_list, [scenes[0].n_rays, 777], "default")
    ref, rc = batch.trace(rays, count=True)
    for waves in (1, 4):
        announce(f"batch of two tiny scenes, {waves} waves per SIMD")
        got, gc = batch.trace(rays, count=True, waves_per_simd=waves)
        torch.cuda.synchronize()
        assert same_bits(got, ref) and same_bits(gc, rc)


@pytest.mark.parametrize("kind", ["default", "alpha"])
def test_tiled_instanced_matches_index_order(env, kind):
    """The instanced traversal with one wave per 8 x 8 tile equals index
    order: hits or occluders, instance ids and counters, into sentinel-filled
    outputs, whole and partial rows of tiles."""
    torch, rtx = env
    wl = W.instanced(300, 256, 120)
    akw = W.instanced_alpha(wl) if kind == "alpha" else {}
    sc = rtx.InstancedScene(wl["blas"], wl["inst_blas"], wl["inst_m"], wl["world_lo"],
                            wl["world_hi"], **akw)
    for n in (wl["rays"].shape[0], wl["rays"].shape[0] - 777, 100):
        rays = torch.from_numpy(wl["rays"][:n].copy()).cuda()
        for any_hit in (False, True):
            announce(f"instanced {kind} n={n} any={any_hit}: tiles of the 256-wide image vs index order")
            ref, rid, rc = sc.trace(rays, kind, any_hit=any_hit, count=True)
            out = (torch.full((n,), 7, dtype=torch.int32, device="cuda") if any_hit
                   else torch.full((n, 4), 7.0, device="cuda"))
            ids = torch.full((n,), 7, dtype=torch.int32, device="cuda")
            got, gid, gc = sc.trace(rays, kind, any_hit=any_hit, count=True, out=out, inst_ids=ids,
                                    image_width=256)
            torch.cuda.synchronize()
            assert same_bits(got, ref) and torch.equal(gid, rid) and same_bits(gc, rc)
