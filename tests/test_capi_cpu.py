"""CPU tests of librtx: symbols, host BVH builder, argument validation.

No test here launches a kernel: the validation cases fail before any HIP
call, and n_rays == 0 returns without a launch.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1912_12786_amd import rtx
from paper_1912_12786_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rtx.h")


@pytest.fixture(scope="module")
def lib():
    return rtx.load_library()


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    fns = header_functions()
    for name in ("rt_bvh_build", "rt_trace_closest", "rt_trace_any", "rt_trace_workspace_bytes",
                 "rt_status_string", "rt_last_error"):
        assert name in fns


def test_every_declared_symbol_is_exported(lib):
    for name in header_functions():
        assert hasattr(lib, name), name
    # and the binding wraps every one of them
    wrapped = {s[0] for s in rtx.SIGNATURES}
    assert set(header_functions()) == wrapped


def test_status_strings(lib):
    for code, name in ((0, "RT_OK"), (-1, "RT_ERR_INVALID_ARG"), (-2, "RT_ERR_MISALIGNED"),
                       (-3, "RT_ERR_UNSUPPORTED"), (-4, "RT_ERR_WORKSPACE"), (-5, "RT_ERR_HIP"),
                       (-6, "RT_ERR_OUT_OF_MEMORY")):
        assert rtx.rt_status_string(code) == name


def test_struct_layout_matches_header(tmp_path):
    """Compiles a probe against include/rtx.h and compares every struct's size
    and field offsets with the ctypes mirrors of the binding."""
    import subprocess
    probe = tmp_path / "probe.c"
    probe.write_text(r"""
#include <stddef.h>
#include <stdio.h>
#include "rtx.h"
#define S(t) printf(#t " %zu\n", sizeof(t));
#define O(t, f) printf(#t "." #f " %zu\n", offsetof(t, f));
int main(void) {
  S(rt_ray) S(rt_hit) S(rt_counters) S(rt_alpha_params) S(rt_procedural_params)
  S(rt_bvh_info) S(rt_scene) S(rt_batch_entry) S(rt_batch_info) S(rt_instance)
  O(rt_instance, object_from_world) O(rt_instance, world_lo) O(rt_instance, world_hi)
  O(rt_batch_entry, n_rays) O(rt_batch_entry, alpha) O(rt_batch_info, max_depth)
  O(rt_alpha_params, textures) O(rt_alpha_params, n_texcoord_prims) O(rt_alpha_params, alpha_min)
  O(rt_bvh_info, root_ref) O(rt_bvh_info, root_lo) O(rt_bvh_info, root_hi)
  O(rt_scene, tris) O(rt_scene, info)
  O(rt_hit, prim_id) O(rt_ray, dx)
  return 0;
}
""")
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(probe), "-o",
                    str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                       check=True).stdout.splitlines())
    got = {k: int(v) for k, v in got.items()}
    assert got["rt_ray"] == 32 and got["rt_hit"] == 16 and got["rt_counters"] == 16
    assert got["rt_hit.prim_id"] == 4 and got["rt_ray.dx"] == 16
    for name, cls in (("rt_alpha_params", rtx.rt_alpha_params),
                      ("rt_procedural_params", rtx.rt_procedural_params),
                      ("rt_bvh_info", rtx.rt_bvh_info), ("rt_scene", rtx.rt_scene),
                      ("rt_batch_entry", rtx.rt_batch_entry), ("rt_batch_info", rtx.rt_batch_info),
                      ("rt_instance", rtx.rt_instance)):
        assert got[name] == C.sizeof(cls), name
        for field, *_ in cls._fields_:
            key = f"{name}.{field}"
            if key in got:
                assert got[key] == getattr(cls, field).offset, key


# ----------------------------------------------------------------------------
# builder parity with the oracle's independent builder
# ----------------------------------------------------------------------------
def decode_product_bvh(nodes_u8, tris_u8, info):
    """Preorder list of (lo, hi, count, first, depth) over all nodes."""
    nf = nodes_u8.view(np.float32).reshape(-1, 16)
    nu = nodes_u8.view(np.uint32).reshape(-1, 16)
    out = []

    def rec(ref, lo, hi, depth):
        cnt, idx = ref >> 29, ref & 0x1FFFFFFF
        out.append((tuple(lo), tuple(hi), cnt, idx if cnt else 0, depth))
        if cnt == 0:
            f = nf[idx]
            rec(int(nu[idx, 12]), f[0:3], f[3:6], depth + 1)
            rec(int(nu[idx, 13]), f[6:9], f[9:12], depth + 1)

    rec(int(info.root_ref), np.array(info.root_lo[:], np.float32),
        np.array(info.root_hi[:], np.float32), 0)
    return out


def decode_oracle_bvh(bvh):
    out = []
    for nd in bvh.nodes:
        cnt = int(nd["count"])
        out.append((tuple(nd["lo"]), tuple(nd["hi"]), cnt, int(nd["first"]) if cnt else 0,
                    int(nd["depth"])))
    return out


def assert_same_bvh(oracle_lib, verts, geom=None):
    nodes, tris, info = rtx.rt_bvh_build(verts, geom)
    ob = oracle_lib.build_bvh(verts)
    prod = decode_product_bvh(nodes, tris, info)
    orc = decode_oracle_bvh(ob)
    assert len(prod) == len(orc)
    for a, b in zip(prod, orc):
        assert np.array_equal(np.array(a[0], np.float32).view(np.uint32),
                              np.array(b[0], np.float32).view(np.uint32))
        assert np.array_equal(np.array(a[1], np.float32).view(np.uint32),
                              np.array(b[1], np.float32).view(np.uint32))
        assert a[2:] == b[2:]
    tu = tris.view(np.uint32).reshape(-1, 12)
    tf = tris.view(np.float32).reshape(-1, 12)
    n = verts.shape[0]
    assert np.array_equal(tu[:, 3], ob.perm)
    v = verts[ob.perm]
    assert np.array_equal(tf[:, 0:3], v[:, 0])
    assert np.array_equal(tf[:, 4:7], v[:, 1] - v[:, 0])
    assert np.array_equal(tf[:, 8:11], v[:, 2] - v[:, 0])
    assert np.all(tu[:, 11] == 0)
    if geom is not None:
        assert np.array_equal(tu[:, 7], geom[ob.perm])
        assert info.max_geom_id == (int(geom.max()) if n else 0)
    assert info.max_depth == ob.max_depth
    assert info.n_nodes == sum(1 for p in prod if p[2] == 0)
    return info


def test_builder_matches_oracle_small(oracle_lib):
    rng = np.random.default_rng(4)
    for n in (1, 3, 4, 5, 8, 17, 100, 1000):
        v = rng.uniform(0, 1, size=(n, 3, 3)).astype(np.float32)
        g = rng.integers(0, 7, size=n).astype(np.uint32)
        assert_same_bvh(oracle_lib, v, g)


def test_builder_matches_oracle_degenerate(oracle_lib):
    v = np.tile(np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0]]], np.float32), (37, 1, 1))
    assert_same_bvh(oracle_lib, v)
    # collinear centroids along one axis only, with duplicates
    x = np.repeat(np.arange(20, dtype=np.float32), 3)
    v = np.zeros((60, 3, 3), np.float32)
    v[:, :, 0] = x[:, None] + np.array([0, 0.5, 0.25], np.float32)
    v[:, 1, 1] = 1.0
    assert_same_bvh(oracle_lib, v)


def test_builder_matches_oracle_tiny_workload(oracle_lib):
    assert_same_bvh(oracle_lib, W.tiny().vertices)


def test_builder_matches_oracle_billboards(oracle_lib):
    wl = W.billboards()
    info = assert_same_bvh(oracle_lib, wl.vertices, wl.geom_ids)
    assert info.max_geom_id == 15


@pytest.mark.slow
def test_builder_matches_oracle_spheres(oracle_lib):
    wl = W.spheres()
    assert_same_bvh(oracle_lib, wl.vertices)


def test_builder_empty_scene():
    nodes, tris, info = rtx.rt_bvh_build(np.zeros((0, 3, 3), np.float32))
    assert info.n_tris == 0 and info.n_nodes == 0 and nodes.size == 0 and tris.size == 0


def test_builder_deterministic():
    v = W.tiny().vertices
    a = rtx.rt_bvh_build(v)
    b = rtx.rt_bvh_build(v)
    assert a[0].tobytes() == b[0].tobytes() and a[1].tobytes() == b[1].tobytes()


def test_buffer_bytes():
    # bounds for any leaf size: n - 1 inner nodes (leaves of one triangle)
    assert rtx.rt_bvh_buffer_bytes(0) == (0, 0)
    assert rtx.rt_bvh_buffer_bytes(1) == (0, 48)
    assert rtx.rt_bvh_buffer_bytes(4) == (3 * 64, 4 * 48)
    assert rtx.rt_bvh_buffer_bytes(5) == (4 * 64, 5 * 48)
    with pytest.raises(rtx.RtxError):
        rtx.rt_bvh_buffer_bytes(1 << 29)


def test_build_rejects_small_buffers(lib):
    v = np.zeros((10, 3, 3), np.float32)
    info = rtx.rt_bvh_info()
    buf = np.zeros(64, np.float32)
    st = lib.rt_bvh_build(v.ctypes.data, None, 10, buf.ctypes.data, 64, buf.ctypes.data, 64,
                          C.byref(info))
    assert st == -1 and "buffer" in rtx.rt_last_error()


# ----------------------------------------------------------------------------
# validation paths (all fail before any HIP call)
# ----------------------------------------------------------------------------
def _fake_scene(n_tris=10, n_nodes=3, root_ref=0, max_depth=3, max_geom=0):
    sc = rtx.rt_scene()
    sc.nodes = 0x10000
    sc.tris = 0x20000
    sc.info.n_tris = n_tris
    sc.info.n_nodes = n_nodes
    sc.info.root_ref = root_ref
    sc.info.max_depth = max_depth
    sc.info.max_geom_id = max_geom
    return sc


def _closest(lib, sc, rays=0x30000, n=100, kind=0, params=None, flags=0, hits=0x40000,
             counters=None, ws=None, wsb=0):
    p = None if params is None else C.cast(C.pointer(params), C.c_void_p)
    return lib.rt_trace_closest(C.byref(sc) if sc is not None else None, rays, n, kind, p, flags,
                                hits, counters, ws, wsb, None)


def test_validation_errors(lib):
    sc = _fake_scene()
    assert _closest(lib, None) == -1
    assert _closest(lib, sc, rays=None) == -1
    assert _closest(lib, sc, n=(1 << 31) + 1) == -1
    assert _closest(lib, sc, rays=0x30004) == -2
    assert _closest(lib, sc, hits=None) == -1
    assert _closest(lib, sc, hits=0x40008) == -2
    assert _closest(lib, sc, kind=7) == -3
    assert _closest(lib, sc, flags=0x10) == -3                       # unknown flag
    assert _closest(lib, sc, flags=rtx.RT_FLAG_LONGEST_FIRST) == -4  # needs its workspace
    assert _closest(lib, sc, flags=6) == -1                          # two runtime modes
    assert _closest(lib, sc, flags=3, counters=0x50000) == -3        # runtime + counting
    assert lib.rt_trace_any(C.byref(sc), 0x30000, 100, 0, None, 2, 0x40000, None, None, 0,
                            None) == -3                              # runtime + any-hit
    assert _closest(lib, sc, flags=rtx.RT_FLAG_COUNT) == -1          # counters missing
    assert _closest(lib, sc, flags=rtx.RT_FLAG_COUNT, counters=0x50004) == -2
    assert _closest(lib, sc, kind=1) == -1                           # alpha params missing
    assert _closest(lib, sc, kind=2) == -1                           # checker params missing
    bad = rtx.rt_procedural_params(0)
    assert _closest(lib, sc, kind=2, params=bad) == -1
    ap = rtx.rt_alpha_params(0x60000, 0x70000, 10, 1, 4, 4, 128)
    sc_g = _fake_scene(max_geom=3)
    assert _closest(lib, sc_g, kind=1, params=ap) == -1              # n_tex <= max geom id
    ap2 = rtx.rt_alpha_params(0x60000, 0x70000, 9, 4, 4, 4, 128)
    assert _closest(lib, sc_g, kind=1, params=ap2) == -1             # texcoords too short
    ap3 = rtx.rt_alpha_params(0x60004, 0x70000, 10, 4, 4, 4, 128)
    assert _closest(lib, sc_g, kind=1, params=ap3) == -2             # texcoords misaligned
    ap4 = rtx.rt_alpha_params(0x60000, 0x70000, 10, 4, 4, 4, 256)
    assert _closest(lib, sc_g, kind=1, params=ap4) == -1             # alpha_min range
    # inconsistent scenes
    assert _closest(lib, _fake_scene(n_nodes=0)) == -1               # inner root without nodes
    assert _closest(lib, _fake_scene(root_ref=(5 << 29))) == -1      # leaf of 5
    assert _closest(lib, _fake_scene(root_ref=(4 << 29) | 8)) == -1  # leaf past the end
    assert _closest(lib, _fake_scene(max_depth=200)) == -1
    sc_mis = _fake_scene()
    sc_mis.tris = 0x20008
    assert _closest(lib, sc_mis) == -2
    # a scene needs workspace (queue head and/or spill space)
    deep = _fake_scene(max_depth=60)
    assert _closest(lib, deep) == -4
    assert "workspace" in rtx.rt_last_error()


def test_multi_validation(lib):
    sc = _fake_scene()
    for k in (0, 9):
        assert lib.rt_trace_multi(C.byref(sc), 0x30000, 100, 0, None, 0, k, 0x40000, 0x50000,
                                  None, None, 0, None) == -1
    # n_hits is required
    assert lib.rt_trace_multi(C.byref(sc), 0x30000, 100, 0, None, 0, 4, 0x40000, None,
                              None, None, 0, None) == -1


def test_batch_pack_layout_and_validation(lib):
    scenes = [_fake_scene(n_tris=10, max_depth=3), _fake_scene(n_tris=0, n_nodes=0),
              _fake_scene(n_tris=20, n_nodes=5, max_depth=7)]
    counts = [100, 0, 37]
    entries = []
    for i, (sc, n) in enumerate(zip(scenes, counts)):
        e = rtx.rt_batch_entry()
        e.scene = sc
        e.scene.nodes = 0x10000 * (i + 1)
        e.scene.info.root_lo[:] = [i, i, i]
        e.n_rays = n
        entries.append(e)
    table, info = rtx.rt_batch_pack(entries, 0)
    assert (info.n_scenes, info.n_rays, info.max_depth, info.kind) == (3, 137, 7, 0)
    assert len(table) == rtx.rt_batch_table_bytes(3)
    u32 = table.view(np.uint32)
    assert u32[0] == 3
    assert u32[16:20].tolist() == [0, 100, 100, 137]          # ray prefix at byte 64
    rec = table[128:].view(np.uint64).reshape(3, 16)            # 128-B records at byte 128
    assert rec[:, 0].tolist() == [0x10000, 0x20000, 0x30000]
    recf = table[128:].view(np.float32).reshape(3, 32)
    assert recf[2, 8:11].tolist() == [2, 2, 2]                  # root_lo
    # an invalid scene is reported with its index
    bad = rtx.rt_batch_entry()
    bad.scene = _fake_scene(n_nodes=0)
    with pytest.raises(rtx.RtxError, match="scene 1"):
        rtx.rt_batch_pack([entries[0], bad], 0)
    # alpha batches validate every entry's alpha data
    with pytest.raises(rtx.RtxError, match="scene 0"):
        rtx.rt_batch_pack([entries[0]], 1)
    ok = rtx.rt_batch_entry()
    ok.scene = _fake_scene()
    ok.alpha = rtx.rt_alpha_params(0x60000, 0x70000, 10, 1, 4, 4, 128)
    t2, i2 = rtx.rt_batch_pack([ok], 1)
    assert i2.kind == 1
    # trace_batch checks the kind against the packed table
    assert lib.rt_trace_batch(0x1000, C.byref(i2), 0x30000, 0, None, 0, 0x40000, None, None, 0,
                              None) == -1
    assert lib.rt_trace_batch(None, C.byref(i2), 0x30000, 1, None, 0, 0x40000, None, None, 0,
                              None) == -1


def test_tlas_build_matches_oracle_box_tree(oracle_lib):
    from paper_1912_12786_amd import workloads as W
    wl = W.instanced(300, 8, 8)
    nodes, tris, info = rtx.rt_tlas_build(wl["inst_blas"], wl["inst_m"], wl["world_lo"],
                                          wl["world_hi"])
    ob = oracle_lib.build_tlas(wl["world_lo"], wl["world_hi"])
    prod = decode_product_bvh(nodes, tris, info)
    orc = decode_oracle_bvh(ob)
    assert len(prod) == len(orc)
    for a, b in zip(prod, orc):
        assert a[0] == b[0] and a[1] == b[1] and a[2:] == b[2:]
    assert np.array_equal(tris.view(np.uint32).reshape(-1, 12)[:, 3], ob.perm)


def test_instance_pack_validation(lib):
    from paper_1912_12786_amd import workloads as W
    wl = W.instanced(5, 8, 8)
    blas = [_fake_scene(), _fake_scene(max_depth=9, max_geom=6), _fake_scene(max_depth=4)]
    table, info = rtx.rt_instance_pack(blas, wl["inst_blas"], wl["inst_m"], wl["world_lo"],
                                       wl["world_hi"])
    assert (info.n_blas, info.n_inst, info.max_blas_depth, info.max_geom_id,
            info.has_texcoords) == (3, 5, 9, 6, 0)
    u32 = table.view(np.uint32)
    assert u32[0] == 3 and u32[1] == 5
    rec = table[64 + 3 * 64:].view(np.float32).reshape(5, 16)
    assert np.array_equal(rec[:, 4:], wl["inst_m"])
    assert np.array_equal(table[64 + 3 * 64:].view(np.uint32).reshape(5, 16)[:, 0], wl["inst_blas"])
    with pytest.raises(rtx.RtxError, match="blas out of range"):
        rtx.rt_instance_pack(blas[:1], np.array([0, 1], np.uint32), wl["inst_m"][:2],
                             wl["world_lo"][:2], wl["world_hi"][:2])
    with pytest.raises(rtx.RtxError, match="bad world box"):
        rtx.rt_tlas_build(np.zeros(1, np.uint32), wl["inst_m"][:1], wl["world_hi"][:1],
                          wl["world_lo"][:1])


def test_instance_pack_texcoords(lib):
    from paper_1912_12786_amd import workloads as W
    wl = W.instanced(5, 8, 8)
    blas = [_fake_scene(), _fake_scene(max_geom=3), _fake_scene(n_tris=0, max_geom=99)]
    tcs = [(0x50000, 10), (0x60000, 12), (None, 0)]
    table, info = rtx.rt_instance_pack(blas, wl["inst_blas"], wl["inst_m"], wl["world_lo"],
                                       wl["world_hi"], tcs)
    # the empty mesh's geom id does not count
    assert info.has_texcoords == 1 and info.max_geom_id == 3
    # blas_record: nodes, tris, root box, root_ref, n_tris, texcoords
    rec = table[64:64 + 3 * 64].view(np.uint64).reshape(3, 8)
    assert list(rec[:, 6]) == [0x50000, 0x60000, 0]
    with pytest.raises(rtx.RtxError, match="bottom-level scene 1: texcoords NULL or covering fewer"):
        rtx.rt_instance_pack(blas, wl["inst_blas"], wl["inst_m"], wl["world_lo"], wl["world_hi"],
                             [(0x50000, 10), (0x60000, 9), (None, 0)])
    with pytest.raises(rtx.RtxError, match="bottom-level scene 0: texcoords NULL"):
        rtx.rt_instance_pack(blas, wl["inst_blas"], wl["inst_m"], wl["world_lo"], wl["world_hi"],
                             [(None, 10), (0x60000, 12), (None, 0)])
    with pytest.raises(rtx.RtxError, match="not 8-byte aligned"):
        rtx.rt_instance_pack(blas, wl["inst_blas"], wl["inst_m"], wl["world_lo"], wl["world_hi"],
                             [(0x50004, 10), (0x60000, 12), (None, 0)])

    # argument checks of the alpha query run before any launch (zero rays)
    tl = _fake_scene()
    ap = rtx.rt_alpha_params()
    ap.textures, ap.n_tex, ap.width, ap.height, ap.alpha_min = 0x70000, 4, 8, 8, 128

    def call(inf, params, kind=rtx.KINDS["alpha"]):
        p = None if params is None else C.cast(C.pointer(params), C.c_void_p)
        return lib.rt_trace_instanced(C.byref(tl), 0x80000, C.byref(inf), None, 0, kind, p, 0, 0,
                                      None, None, None, None, 0, None)

    assert call(info, ap) == 0
    _, bare = rtx.rt_instance_pack(blas, wl["inst_blas"], wl["inst_m"], wl["world_lo"],
                                   wl["world_hi"])
    assert call(bare, ap) == -1
    assert b"without texture coordinates" in lib.rt_last_error()
    ap.n_tex = 3
    assert call(info, ap) == -1
    assert b"exceeds the texture count" in lib.rt_last_error()
    ap.n_tex = 4
    assert call(info, None) == -1
    ap.alpha_min = 256
    assert call(info, ap) == -1
    assert lib.rt_trace_instanced(C.byref(tl), 0x80000, None, None, 0, 0, None, 0, 0, None, None,
                                  None, None, 0, None) == -1


def test_zero_rays_is_a_no_op(lib):
    sc = _fake_scene()
    assert _closest(lib, sc, rays=None, n=0, hits=None) == 0
    assert lib.rt_trace_any(C.byref(sc), None, 0, 0, None, 0, None, None, None, 0, None) == 0


def test_workspace_bytes(lib):
    shapes = rtx.rt_launch_shapes()
    assert len(shapes) >= 1
    for i, (block, slots, chunk, queue) in enumerate(shapes):
        f = rtx.RT_FLAG_SHAPE(i)
        assert rtx.shape_flag((block, slots, chunk, queue)) == f
        for n in (1000, 3_000_000):
            b = rtx.rt_trace_workspace_bytes(_fake_scene(max_depth=20), n, f)
            waves = (n + chunk - 1) // chunk
            if queue:
                waves = min(waves, 256 * 32)
            threads = (waves * 64 + block - 1) // block * block
            assert b == (1024 if queue else 0) + max(0, 20 - (slots - 1)) * threads * 8
            # shallow scenes need no spill space
            shallow = rtx.rt_trace_workspace_bytes(_fake_scene(max_depth=slots - 1), n, f)
            assert shallow == (1024 if queue else 0)
    # the default field (0) is the first shape
    assert rtx.rt_trace_workspace_bytes(_fake_scene(max_depth=20), 5000) == \
        rtx.rt_trace_workspace_bytes(_fake_scene(max_depth=20), 5000, rtx.RT_FLAG_SHAPE(0))
    # an index past the table is refused, here and by the trace calls
    with pytest.raises(rtx.RtxError, match="launch shape"):
        rtx.rt_trace_workspace_bytes(_fake_scene(max_depth=20), 5000, rtx.RT_FLAG_SHAPE(len(shapes)))
    with pytest.raises(rtx.RtxError, match="not compiled in"):
        rtx.shape_flag((3, 3, 3, 3))
    # every flag a trace call accepts is accepted here, with the same size
    sc = _fake_scene(max_depth=20)
    base = rtx.rt_trace_workspace_bytes(sc, 5000)
    for flags in (rtx.RT_FLAG_COUNT, rtx.RT_FLAG_RUNTIME_SWITCH, rtx.RT_FLAG_RUNTIME_CALL):
        assert rtx.rt_trace_workspace_bytes(sc, 5000, flags) == base
    with pytest.raises(rtx.RtxError):
        rtx.rt_trace_workspace_bytes(sc, 5000, 1 << 7)


def test_binding_fails_loudly_without_library(tmp_path):
    import importlib
    with pytest.raises(ImportError):
        # a fresh load from a path with no library must raise, not fall back
        saved = rtx._lib
        try:
            rtx._lib = None
            rtx.load_library(str(tmp_path / "librtx.so"))
        finally:
            rtx._lib = saved
    importlib.invalidate_caches()


def test_custom_intersector_library_loads_and_validates(lib):
    """The user-defined intersector library (compiled against the traversal
    template) loads, exports its entry points, sizes its workspace like the
    library's default shape, and validates arguments without a GPU."""
    from tests.custom import binding
    cl = binding.load()
    sc = _fake_scene(max_depth=20)
    assert cl.prim_mask_workspace_bytes(C.byref(sc), 5000) == rtx.rt_trace_workspace_bytes(sc, 5000)
    # zero rays: nothing to do
    assert cl.prim_mask_trace(C.byref(sc), None, 0, 0x10, None, None, None, 0, None) == 0
    # status codes of include/rtx.h: -1 invalid argument, -2 misaligned, -4 workspace
    # no mask for a non-empty scene
    assert cl.prim_mask_trace(C.byref(sc), 0x30000, 10, None, 0x40000, None, 0x50000, 1 << 20,
                              None) == -1
    # misaligned output, too-small workspace
    assert cl.prim_mask_trace(C.byref(sc), 0x30000, 10, 0x10, 0x40008, None, 0x50000, 1 << 20,
                              None) == -2
    assert cl.prim_mask_trace(C.byref(sc), 0x30000, 10, 0x10, 0x40000, None, 0x50000, 16,
                              None) == -4


# ----------------------------------------------------------------------------
# 32-byte node layout
# ----------------------------------------------------------------------------
def _q8_scenes():
    from paper_1912_12786_amd import workloads as W
    rng = np.random.default_rng(11)
    flat = W.random_triangles(300, 12, side=0.2, box=(-3.0, 3.0)).copy()
    flat[::3, :, 1] = flat[::3, :1, 1]                      # zero extent on y
    return {"tiny": W.tiny().vertices,
            "billboards": W.billboards(3000).vertices,
            "negative_flat": flat,
            "far": (rng.uniform(-1, 1, size=(500, 3, 3)) * 0.01 + 5e3).astype(np.float32)}


@pytest.mark.parametrize("name", ["tiny", "billboards", "negative_flat", "far"])
def test_compress_matches_oracle_quantizer(lib, oracle_lib, name):
    """The product's 32-byte nodes equal the oracle's quantization of its own
    (identical) BVH word for word: frames, 8-bit coordinates, references."""
    v = _q8_scenes()[name]
    nodes, tris, info = rtx.rt_bvh_build(v)
    q, qi = rtx.rt_bvh_compress(nodes, info)
    assert qi.layout == 1 and qi.n_nodes == info.n_nodes and qi.root_ref == info.root_ref
    b = oracle_lib.build_bvh(v)
    Q = oracle_lib.quantize(b)
    inner = np.nonzero(b.nodes["count"] == 0)[0]
    assert inner.size == info.n_nodes
    w = q.view(np.uint32).reshape(-1, 8)
    assert np.array_equal(w[:, :3], Q["frames"][inner])
    assert np.array_equal(w[:, 3:6].copy().view(np.uint8).reshape(-1, 12), Q["q"][inner])
    assert np.array_equal(w[:, 6:8], nodes.view(np.uint32).reshape(-1, 16)[:, 12:14])


def test_compress_validation(lib):
    v = _q8_scenes()["tiny"]
    nodes, tris, info = rtx.rt_bvh_build(v)
    q, qi = rtx.rt_bvh_compress(nodes, info)
    with pytest.raises(rtx.RtxError, match="not RT_LAYOUT_F32"):
        rtx.rt_bvh_compress(nodes, qi)
    bad = nodes.copy()
    bad.view(np.float32)[3] = np.inf                         # hi0.x of node 0
    with pytest.raises(rtx.RtxError, match="not finite"):
        rtx.rt_bvh_compress(bad, info)
    empty = rtx.rt_bvh_info()
    _, ei = rtx.rt_bvh_compress(np.zeros(0, np.uint8), empty)
    assert ei.layout == 1 and ei.n_nodes == 0
    sc = _fake_scene()
    sc.info.layout = 4
    assert _closest(lib, sc) == -1
    assert b"unknown scene node layout" in lib.rt_last_error()
    sc.info.layout = 1
    assert _closest(lib, sc, n=0) == 0
    # instancing takes float32-box scenes only
    from paper_1912_12786_amd import workloads as W
    wl = W.instanced(3, 8, 8)
    with pytest.raises(rtx.RtxError, match="RT_LAYOUT_F32"):
        rtx.rt_instance_pack([_fake_scene(), sc], np.zeros(3, np.uint32), wl["inst_m"][:3],
                             wl["world_lo"][:3], wl["world_hi"][:3])


# ----------------------------------------------------------------------------
# leaf size (rt_bvh_build_ex)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("max_leaf", [1, 2, 3, 7])
@pytest.mark.parametrize("name", ["tiny", "negative_flat"])
def test_leaf_size_builds_match_oracle(lib, oracle_lib, name, max_leaf):
    """The product's BVH with leaves of at most max_leaf triangles equals the
    oracle's independent build with the same limit, node for node."""
    v = _q8_scenes()[name]
    nodes, tris, info = rtx.rt_bvh_build(v, max_leaf=max_leaf)
    assert info.max_leaf == max_leaf
    ob = oracle_lib.build_bvh(v, max_leaf=max_leaf)
    prod = decode_product_bvh(nodes, tris, info)
    orc = decode_oracle_bvh(ob)
    assert len(prod) == len(orc)
    for a, b in zip(prod, orc):
        for k in (0, 1):
            assert np.array_equal(np.array(a[k], np.float32).view(np.uint32),
                                  np.array(b[k], np.float32).view(np.uint32))
        assert a[2:] == b[2:]
    assert np.array_equal(tris.view(np.uint32).reshape(-1, 12)[:, 3], ob.perm)
    counts = ob.nodes["count"]
    assert counts.max() <= max_leaf and (counts > 0).sum() >= v.shape[0] / max_leaf


def test_leaf_size_validation(lib):
    v = np.zeros((3, 3, 3), np.float32)
    for bad in (0, 8):
        with pytest.raises(rtx.RtxError, match="max_leaf"):
            rtx.rt_bvh_build(v, max_leaf=bad)
    # a root leaf of 7 triangles is a valid scene
    v7 = np.random.default_rng(1).uniform(0, 1, size=(7, 3, 3)).astype(np.float32)
    nodes, tris, info = rtx.rt_bvh_build(v7, max_leaf=7)
    assert info.n_nodes == 0 and info.root_ref >> 29 == 7
    sc = _fake_scene(n_tris=7, n_nodes=0, root_ref=(7 << 29))
    assert _closest(lib, sc, n=0) == -1              # hand-made info: limit 4
    sc.info.max_leaf = 7
    assert _closest(lib, sc, n=0) == 0


def test_noalloc_rejects_before_any_device_work(lib):
    """rt_trace_closest_noalloc validates like rt_trace_closest and refuses a
    call whose workspace exceeds its fixed scratch, all before a HIP call."""
    def call(sc, n=100, flags=0, rays=0x30000, hits=0x40000, counters=None):
        return lib.rt_trace_closest_noalloc(C.byref(sc) if sc is not None else None, rays, n, 0,
                                            None, flags, hits, counters, None)
    sc = _fake_scene()
    assert call(None) == -1
    assert call(sc, rays=None) == -1
    assert call(sc, hits=0x40008) == -2
    assert call(sc, flags=rtx.RT_FLAG_COUNT) == -1
    assert call(sc, n=(1 << 31) + 1) == -1
    assert call(sc, n=0) == 0                      # no rays: no launch, no scratch lookup
    assert call(sc, flags=rtx.RT_FLAG_SHAPE(len(rtx.rt_launch_shapes()))) == -3
    # the default shape's spill space at the full persistent grid: 4 MiB per
    # stack level beyond the 7 in LDS, so max_depth 22 fits and 23 does not
    full = 3_000_000
    for depth, ok in ((22, True), (23, False), (100, False)):
        need = rtx.rt_trace_workspace_bytes(_fake_scene(max_depth=depth), full)
        assert (need <= rtx.RT_NOALLOC_SCRATCH_BYTES) == ok, (depth, need)
    assert call(_fake_scene(max_depth=23), n=full) == -4
    assert "fixed scratch" in rtx.rt_last_error()
    # a deep scene still fits with fewer rays per call
    need = rtx.rt_trace_workspace_bytes(_fake_scene(max_depth=100), 20_000)
    assert need <= rtx.RT_NOALLOC_SCRATCH_BYTES


# ----------------------------------------------------------------------------
# four-wide nodes (rt_bvh_widen) against the oracle's collapse
# ----------------------------------------------------------------------------
def decode_product_wide(nodes_u8, info):
    """Preorder list of (child count, [(lo, hi, leaf count, leaf first)]) of
    the wide nodes, leaf firsts as triangle-record positions."""
    nf = nodes_u8.view(np.float32).reshape(-1, 32)
    nu = nodes_u8.view(np.uint32).reshape(-1, 32)
    out = []

    def rec(w):
        refs = [int(x) for x in nu[w, 24:28]]
        k = sum(1 for r in refs if r != rtx.RT_WIDE_EMPTY_REF)
        assert all(r == rtx.RT_WIDE_EMPTY_REF for r in refs[k:]), "unused slots must be last"
        assert np.all(nu[w, 28:32] == 0)
        kids = []
        for c in range(k):
            lo = nf[w, [c, 8 + c, 16 + c]]
            hi = nf[w, [4 + c, 12 + c, 20 + c]]
            cnt, idx = refs[c] >> 29, refs[c] & 0x1FFFFFFF
            kids.append((lo.view(np.uint32).tolist(), hi.view(np.uint32).tolist(), cnt,
                         idx if cnt else None))
        for c in range(k, 4):
            assert np.all(nu[w, [c, 4 + c, 8 + c, 12 + c, 16 + c, 20 + c]] == 0)
        out.append((k, kids))
        for c in range(k):
            if refs[c] >> 29 == 0:
                assert refs[c] > w, "wide nodes must be numbered in preorder"
                rec(refs[c])

    if info.n_nodes:
        rec(0)
    return out


def decode_oracle_wide(bvh, w):
    nodes = bvh.nodes
    out = []
    for h in w["order"]:
        e = w["wide"][h]
        kids = []
        for c in e["child"][: e["n"]]:
            nd = nodes[int(c)]
            cnt = int(nd["count"])
            kids.append((nd["lo"].astype(np.float32).view(np.uint32).tolist(),
                         nd["hi"].astype(np.float32).view(np.uint32).tolist(), cnt,
                         int(nd["first"]) if cnt else None))
        out.append((int(e["n"]), kids))
    return out


def assert_same_wide(oracle_lib, verts, max_leaf):
    nodes, tris, info = rtx.rt_bvh_build(verts, max_leaf=max_leaf)
    wn, winfo = rtx.rt_bvh_widen(nodes, info)
    ob = oracle_lib.build_bvh(verts, max_leaf=max_leaf)
    ow = oracle_lib.widen(ob)
    assert winfo.layout == rtx.LAYOUTS["wide4"]
    assert winfo.n_nodes == len(ow["order"])
    assert winfo.max_depth == ow["stack_bound"]
    assert decode_product_wide(wn, winfo) == decode_oracle_wide(ob, ow)
    if info.root_ref >> 29:
        assert winfo.root_ref == info.root_ref and winfo.n_nodes == 0
    else:
        assert winfo.root_ref == 0
    for f in ("n_tris", "max_geom_id", "max_leaf"):
        assert getattr(winfo, f) == getattr(info, f)
    assert list(winfo.root_lo) == list(info.root_lo) and list(winfo.root_hi) == list(info.root_hi)
    return winfo


def test_widen_matches_oracle(oracle_lib):
    rng = np.random.default_rng(9)
    for n in (1, 3, 5, 8, 9, 17, 100, 1000):
        for ml in (1, 2, 4):
            v = rng.uniform(0, 1, size=(n, 3, 3)).astype(np.float32)
            assert_same_wide(oracle_lib, v, ml)
    assert_same_wide(oracle_lib, W.tiny().vertices, 4)


def test_widen_matches_oracle_billboards(oracle_lib):
    wl = W.billboards()
    info = assert_same_wide(oracle_lib, wl.vertices, 2)
    assert 0 < info.max_depth < 128


def test_widen_validation(lib):
    info = rtx.rt_bvh_info()
    info.layout = 1
    out = rtx.rt_bvh_info()
    assert lib.rt_bvh_widen(None, C.byref(info), None, 0, C.byref(out)) == -1   # not float32 nodes
    nodes, tris, binfo = rtx.rt_bvh_build(W.tiny().vertices)
    buf = np.zeros(16, np.uint8)
    assert lib.rt_bvh_widen(nodes.ctypes.data, C.byref(binfo), buf.ctypes.data, 16,
                            C.byref(out)) == -1                                  # out too small
    assert "smaller" in rtx.rt_last_error()
    assert lib.rt_bvh_widen(None, None, None, 0, None) == -1
    # a wide scene is accepted by the trace calls' validation (it fails later on
    # the fake device pointers only when launched, which the CPU never does)
    sc = _fake_scene(max_depth=30)
    sc.info.layout = rtx.LAYOUTS["wide4"]
    need = rtx.rt_trace_workspace_bytes(sc, 1000)
    assert need > 1024
    # runtime dispatch is compiled for binary float32 nodes only
    assert _closest(lib, sc, flags=rtx.RT_FLAG_RUNTIME_SWITCH, ws=0x80000, wsb=need) == -3


def test_tile_flag(lib):
    assert rtx.tile_flag(None) == 0 and rtx.tile_flag(1920) == 240 << 16
    for bad in (12, 32768, -8):
        with pytest.raises(ValueError):
            rtx.tile_flag(bad)
    # accepted by the single-scene calls' validation, refused by the batched
    # and instanced launches
    sc = _fake_scene()
    assert _closest(lib, sc, n=0, flags=rtx.tile_flag(1920)) == 0
    info = rtx.rt_batch_info()
    assert lib.rt_trace_batch(0x10000, C.byref(info), 0x30000, 0, None, rtx.tile_flag(1920),
                              0x40000, None, None, 0, None) == -3


def test_longest_first_workspace(lib):
    """The longest-path-first schedule adds a key and an order entry per
    chunk plus a row of 64 bucket counts per 256 chunks, rounded to 16."""
    sc = _fake_scene(max_depth=3)
    for shape in rtx.rt_launch_shapes():
        f = rtx.shape_flag(tuple(shape))
        for n in (1, 64, 65, 256 * 64, 256 * 64 + 1, 2_073_600):
            plain = rtx.rt_trace_workspace_bytes(sc, n, f)
            lf = rtx.rt_trace_workspace_bytes(sc, n, f | rtx.RT_FLAG_LONGEST_FIRST)
            chunks = -(-n // shape[2])
            rows = -(-chunks // 256)
            assert lf - plain == (8 * chunks + 256 * rows + 15) // 16 * 16
    info = rtx.rt_batch_info()
    assert lib.rt_trace_batch(0x10000, C.byref(info), 0x30000, 0, None, rtx.RT_FLAG_LONGEST_FIRST,
                              0x40000, None, None, 0, None) == -3


def test_waves_per_simd_flag(lib, tmp_path):
    """The persistent-grid cap (RT_FLAG_WAVES_PER_SIMD): the header's field
    and default equal the binding's; every value passes flag validation (the
    call then stops only at its missing workspace) and leaves the workspace
    size unchanged; the binding refuses values outside 1..15."""
    import subprocess
    probe = tmp_path / "waves.c"
    probe.write_text(r"""
#include <stdio.h>
#include "rtx.h"
int main(void) {
  printf("%u %u %u %u\n", RT_FLAG_WAVES_SHIFT, RT_FLAG_WAVES_MASK, RT_DEFAULT_WAVES_PER_SIMD,
         RT_FLAG_WAVES_PER_SIMD(5));
  return 0;
}
""")
    exe = tmp_path / "waves"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(probe), "-o",
                    str(exe)], check=True)
    vals = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    assert vals == [rtx.RT_FLAG_WAVES_SHIFT, rtx.RT_FLAG_WAVES_MASK,
                    rtx.RT_DEFAULT_WAVES_PER_SIMD, rtx.waves_flag(5)]
    sc = _fake_scene(max_depth=3)
    for w in range(16):
        f = w << rtx.RT_FLAG_WAVES_SHIFT
        assert _closest(lib, sc, flags=f) == -4
        for n in (1, 65, 2_073_600):
            assert rtx.rt_trace_workspace_bytes(sc, n, f) == rtx.rt_trace_workspace_bytes(sc, n, 0)
    info = rtx.rt_batch_info()
    info.n_rays, info.max_depth = 100_000, 20
    for w in range(16):
        assert (rtx.rt_trace_batch_workspace_bytes(info, w << rtx.RT_FLAG_WAVES_SHIFT)
                == rtx.rt_trace_batch_workspace_bytes(info, 0))
    assert rtx.waves_flag(None) == 0 and rtx.waves_flag(0) == 0
    for bad in (16, -1):
        with pytest.raises(ValueError):
            rtx.waves_flag(bad)


@pytest.mark.parametrize("name", ["tiny", "billboards", "negative_flat", "far"])
def test_pack_matches_oracle(lib, oracle_lib, name):
    """The product's 48-byte nodes equal the oracle's packing of its own
    (identical) BVH word for word, and their gathered bytes are the 64-byte
    nodes' references."""
    v = _q8_scenes()[name]
    for max_leaf in (1, 2, 4):
        nodes, tris, info = rtx.rt_bvh_build(v, None, max_leaf)
        p, pi = rtx.rt_bvh_pack(nodes, info)
        assert pi.layout == 3 and pi.n_nodes == info.n_nodes and pi.root_ref == info.root_ref
        b = oracle_lib.build_bvh(v, max_leaf=max_leaf)
        P = oracle_lib.pack(b)
        inner = np.nonzero(b.nodes["count"] == 0)[0]
        assert inner.size == info.n_nodes
        w = p.view(np.uint32).reshape(-1, 12)
        assert np.array_equal(w, P["box"][inner].view(np.uint32))
        refs = nodes.view(np.uint32).reshape(-1, 16)[:, 12:14]
        assert np.array_equal(refs, P["refs"][inner])


def test_pack_validation(lib):
    v = _q8_scenes()["tiny"]
    nodes, tris, info = rtx.rt_bvh_build(v)
    p, pi = rtx.rt_bvh_pack(nodes, info)
    with pytest.raises(rtx.RtxError, match="not RT_LAYOUT_F32"):
        rtx.rt_bvh_pack(nodes, pi)
    bad = nodes.copy()
    bad.view(np.float32)[3] = np.inf                          # hi0.x of node 0
    with pytest.raises(rtx.RtxError, match="not finite"):
        rtx.rt_bvh_pack(bad, info)
    # hi0.x 15 patterns below +FLT_MAX must carry ref0's top byte (< 0xF0):
    # its upward walk would reach +infinity
    edge = nodes.copy()
    edge.view(np.uint32)[3] = 0x7F7FFFF0
    assert int(edge.view(np.uint32)[12]) >> 24 < 0xF0
    with pytest.raises(rtx.RtxError, match="float range"):
        rtx.rt_bvh_pack(edge, info)
    empty = rtx.rt_bvh_info()
    _, ei = rtx.rt_bvh_pack(np.zeros(0, np.uint8), empty)
    assert ei.layout == 3 and ei.n_nodes == 0


def test_refit_plan(lib):
    """rt_bvh_refit_plan: every inner node's parent and slot and its depth
    (recomputed here from the decoded tree), the top flag exactly on the nodes
    whose preorder subtree range leaves their block of 1024 numbers, and the
    list of those nodes; a root leaf has no plan; other layouts and trees
    with a reference back up are refused."""
    from paper_1912_12786_amd import workloads as W
    for verts, leaf in ((W.tiny().vertices, 2), (W.billboards(3000).vertices, 1),
                        (W.tiny().vertices[:200], 1), (W.tiny().vertices[:3], 4)):
        nodes, tris, info = rtx.rt_bvh_build(verts, None, leaf)
        plan, n_top = rtx.rt_bvh_refit_plan(nodes, info)
        n = info.n_nodes
        if n == 0:
            assert plan.size == 0 and n_top == 0
            continue
        nu = nodes.view(np.uint32).reshape(-1, 16)
        parent = np.full(n, 0xFFFFFFFF, np.uint64)
        depth = np.zeros(n, np.int64)
        for k in range(n):
            for c in (0, 1):
                ref = int(nu[k, 12 + c])
                if ref >> 29 == 0:
                    parent[ref] = 2 * k + c
                    depth[ref] = depth[k] + 1
        size = np.ones(n, np.int64)
        for k in range(n - 1, 0, -1):
            size[int(parent[k]) >> 1] += size[k]
        top = (np.arange(n) + size) > (np.arange(n) // 1024 + 1) * 1024
        assert plan.size == 2 * n + n_top
        assert np.array_equal(plan[:n], parent.astype(np.uint32))
        assert np.array_equal(plan[n:2 * n] & 0x7FFFFFFF, depth.astype(np.uint32))
        assert np.array_equal((plan[n:2 * n] >> 31).astype(bool), top)
        assert np.array_equal(plan[2 * n:], np.nonzero(top)[0].astype(np.uint32))
        assert (n_top > 0) == (n > 1024)
    nodes, tris, info = rtx.rt_bvh_build(W.tiny().vertices)
    q, qi = rtx.rt_bvh_compress(nodes, info)
    with pytest.raises(rtx.RtxError, match="RT_LAYOUT_F32"):
        rtx.rt_bvh_refit_plan(nodes, qi)
    # a child reference pointing back up is refused
    bad = nodes.copy()
    bu = bad.view(np.uint32).reshape(-1, 16)
    inner = [c for c in (12, 13) if bu[1, c] >> 29 == 0]
    bu[1, inner[0] if inner else 12] = 0
    with pytest.raises(rtx.RtxError, match="later node"):
        rtx.rt_bvh_refit_plan(bad, info)


def test_refit_validation(lib):
    """Argument errors of rt_bvh_refit are found before any device work."""
    sc = _fake_scene(n_tris=3000, n_nodes=1300, max_depth=3)
    f = lib.rt_bvh_refit
    P, V, F, R = 0x10000, 0x30000, 0x40000, 0x50000
    assert f(C.byref(sc), P, 5, None, 10, F, R, None) == -1            # vertices NULL
    assert f(C.byref(sc), P, 5, V, 10, F, None, None) == -1            # root box NULL
    assert f(C.byref(sc), P, 5, V + 2, 10, F, R, None) == -2           # misaligned
    assert f(C.byref(sc), None, 5, V, 10, F, R, None) == -1            # inner root, no plan
    assert f(C.byref(sc), P + 2, 5, V, 10, F, R, None) == -2           # misaligned plan
    assert f(C.byref(sc), P, 1301, V, 10, F, R, None) == -1            # n_top > n_nodes
    assert f(C.byref(sc), P, 0, V, 10, F, R, None) == -1               # > 1024 nodes, no top
    sc.info.root_ref = 1
    assert f(C.byref(sc), P, 5, V, 10, F, R, None) == -1               # root not node 0
    sc.info.root_ref = 0
    sc.info.layout = 1
    assert f(C.byref(sc), P, 5, V, 10, F, R, None) == -3               # another layout
