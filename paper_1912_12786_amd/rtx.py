"""Python binding of librtx (ctypes).

Functions named ``rt_*`` mirror the C ABI in ``include/rtx.h`` one to one and
only marshal arguments; every step of the traversal runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  The helpers below
them (:class:`Scene`, :func:`trace`) allocate outputs with torch and call the
same entry points.

There is no fallback: if ``librtx.so`` is missing or fails to load, every
entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtx.so")

RT_OK = 0
RT_ERR_UNSUPPORTED = -3
RT_MISS = 0xFFFFFFFF
RT_FLAG_COUNT = 1
RT_FLAG_RUNTIME_SWITCH = 2
RT_FLAG_RUNTIME_CALL = 4
RT_FLAG_LONGEST_FIRST = 8
RT_FLAG_SHAPE_SHIFT = 8
RT_FLAG_SHAPE_MASK = 0xFF00
RT_FLAG_TILE_SHIFT = 16
RT_FLAG_TILE_MASK = 0x0FFF0000
RT_FLAG_WAVES_SHIFT = 28
RT_FLAG_WAVES_MASK = 0xF0000000
RT_DEFAULT_WAVES_PER_SIMD = 7
RT_NODE_BYTES = 64
RT_NODE_BYTES_Q8 = 32
RT_NODE_BYTES_WIDE4 = 128
RT_NODE_BYTES_F32P = 48
RT_WIDE_EMPTY_REF = 0xFFFFFFFF
RT_TRI_BYTES = 48
RT_NOALLOC_SCRATCH_BYTES = 64 << 20
LAYOUTS = {"f32": 0, "q8": 1, "wide4": 2, "f32p": 3}
KINDS = {"default": 0, "alpha": 1, "procedural": 2}


class RtxError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {_status_name(status)}: {detail}")
        self.status = status


class rt_alpha_params(C.Structure):
    _fields_ = [("texcoords", C.c_void_p), ("textures", C.c_void_p),
                ("n_texcoord_prims", C.c_uint32), ("n_tex", C.c_uint32),
                ("width", C.c_uint32), ("height", C.c_uint32), ("alpha_min", C.c_uint32)]


class rt_procedural_params(C.Structure):
    _fields_ = [("checker_n", C.c_uint32)]


class rt_bvh_info(C.Structure):
    _fields_ = [("n_tris", C.c_uint32), ("n_nodes", C.c_uint32), ("max_depth", C.c_uint32),
                ("max_geom_id", C.c_uint32), ("root_ref", C.c_uint32),
                ("root_lo", C.c_float * 3), ("root_hi", C.c_float * 3), ("layout", C.c_uint32),
                ("max_leaf", C.c_uint32)]


class rt_build_params(C.Structure):
    _fields_ = [("max_leaf", C.c_uint32)]


class rt_scene(C.Structure):
    _fields_ = [("nodes", C.c_void_p), ("tris", C.c_void_p), ("info", rt_bvh_info)]


class rt_instance(C.Structure):
    _fields_ = [("blas", C.c_uint32), ("object_from_world", C.c_float * 12),
                ("world_lo", C.c_float * 3), ("world_hi", C.c_float * 3)]


class rt_mesh_texcoords(C.Structure):
    _fields_ = [("texcoords", C.c_void_p), ("n_prims", C.c_uint32)]


class rt_instance_info(C.Structure):
    _fields_ = [("n_blas", C.c_uint32), ("n_inst", C.c_uint32), ("max_blas_depth", C.c_uint32),
                ("max_geom_id", C.c_uint32), ("has_texcoords", C.c_uint32)]


class rt_batch_entry(C.Structure):
    _fields_ = [("scene", rt_scene), ("n_rays", C.c_uint32), ("alpha", rt_alpha_params)]


class rt_batch_info(C.Structure):
    _fields_ = [("n_scenes", C.c_uint32), ("n_rays", C.c_uint32), ("max_depth", C.c_uint32),
                ("kind", C.c_uint32), ("layout", C.c_uint32)]


_lib = None

# (name, restype, argtypes) of every entry point declared in include/rtx.h
_P, _U32, _SZ = C.c_void_p, C.c_uint32, C.c_size_t
SIGNATURES = [
    ("rt_bvh_buffer_bytes", C.c_int, [_U32, C.POINTER(_SZ), C.POINTER(_SZ)]),
    ("rt_bvh_build", C.c_int, [_P, _P, _U32, _P, _SZ, _P, _SZ, C.POINTER(rt_bvh_info)]),
    ("rt_bvh_build_ex", C.c_int, [_P, _P, _U32, C.POINTER(rt_build_params), _P, _SZ, _P, _SZ,
                                  C.POINTER(rt_bvh_info)]),
    ("rt_bvh_compress", C.c_int, [_P, C.POINTER(rt_bvh_info), _P, _SZ, C.POINTER(rt_bvh_info)]),
    ("rt_bvh_widen", C.c_int, [_P, C.POINTER(rt_bvh_info), _P, _SZ, C.POINTER(rt_bvh_info)]),
    ("rt_bvh_pack", C.c_int, [_P, C.POINTER(rt_bvh_info), _P, _SZ, C.POINTER(rt_bvh_info)]),
    ("rt_bvh_refit_plan", C.c_int, [_P, C.POINTER(rt_bvh_info), _P, _SZ, C.POINTER(C.c_uint32)]),
    ("rt_bvh_refit", C.c_int, [C.POINTER(rt_scene), _P, _U32, _P, _U32, _P, _P, _P]),
    ("rt_trace_workspace_bytes", C.c_int, [C.POINTER(rt_scene), _U32, _U32, C.POINTER(_SZ)]),
    ("rt_trace_closest", C.c_int, [C.POINTER(rt_scene), _P, _U32, C.c_int, _P, _U32, _P, _P, _P,
                                   _SZ, _P]),
    ("rt_trace_closest_noalloc", C.c_int, [C.POINTER(rt_scene), _P, _U32, C.c_int, _P, _U32,
                                           _P, _P, _P]),
    ("rt_trace_any", C.c_int, [C.POINTER(rt_scene), _P, _U32, C.c_int, _P, _U32, _P, _P, _P,
                               _SZ, _P]),
    ("rt_batch_table_bytes", C.c_int, [_U32, C.POINTER(_SZ)]),
    ("rt_batch_pack", C.c_int, [_P, _U32, C.c_int, _P, _SZ, C.POINTER(rt_batch_info)]),
    ("rt_trace_batch_workspace_bytes", C.c_int, [C.POINTER(rt_batch_info), _U32, C.POINTER(_SZ)]),
    ("rt_trace_batch", C.c_int, [_P, C.POINTER(rt_batch_info), _P, C.c_int, _P, _U32, _P, _P, _P,
                                 _SZ, _P]),
    ("rt_tlas_build", C.c_int, [_P, _U32, _P, _SZ, _P, _SZ, C.POINTER(rt_bvh_info)]),
    ("rt_instance_table_bytes", C.c_int, [_U32, _U32, C.POINTER(_SZ)]),
    ("rt_instance_pack", C.c_int, [_P, _P, _U32, _P, _U32, _P, _SZ, C.POINTER(rt_instance_info)]),
    ("rt_trace_instanced_workspace_bytes", C.c_int, [C.POINTER(rt_scene),
                                                     C.POINTER(rt_instance_info), _U32, _U32,
                                                     C.POINTER(_SZ)]),
    ("rt_trace_instanced", C.c_int, [C.POINTER(rt_scene), _P, C.POINTER(rt_instance_info), _P,
                                     _U32, C.c_int, _P, _U32, C.c_int, _P, _P, _P, _P, _SZ, _P]),
    ("rt_trace_multi", C.c_int, [C.POINTER(rt_scene), _P, _U32, C.c_int, _P, _U32, _U32, _P, _P,
                                 _P, _P, _SZ, _P]),
    ("rt_hit_backward", C.c_int, [_P, _P, _P, _U32, _P, _U32, _P, _U32, _P, _P, _P]),
    ("rt_launch_shapes", C.c_uint32, [_P, _P, _P, _P, _U32]),
    ("rt_status_string", C.c_char_p, [C.c_int]),
    ("rt_last_error", C.c_char_p, []),
]


def load_library(path: str = LIB_PATH):
    """Loads librtx.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"librtx.so not found at {path}; build it with "
                              f"`python -m paper_1912_12786_amd.build`")
        lib = C.CDLL(path)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _status_name(s: int) -> str:
    try:
        return load_library().rt_status_string(s).decode()
    except Exception:  # pragma: no cover - only used while formatting errors
        return str(s)


def _check(status: int, where: str):
    if status != RT_OK:
        detail = load_library().rt_last_error().decode()
        raise RtxError(status, where, detail)


# ----------------------------------------------------------------------------
# one-to-one wrappers of the C ABI
# ----------------------------------------------------------------------------
def rt_bvh_buffer_bytes(n_tris: int):
    lib = load_library()
    nb, tb = C.c_size_t(), C.c_size_t()
    _check(lib.rt_bvh_buffer_bytes(n_tris, C.byref(nb), C.byref(tb)), "rt_bvh_buffer_bytes")
    return nb.value, tb.value


def rt_bvh_build(vertices: np.ndarray, geom_ids: np.ndarray | None = None, max_leaf: int = 4):
    """Host BVH build (rt_bvh_build_ex; leaves of at most ``max_leaf``
    triangles).  Returns ``(nodes, tris, info)``: uint8 arrays holding
    ``info.n_nodes`` 64-byte node records and ``n_tris`` 48-byte triangle
    records, and the filled ``rt_bvh_info``."""
    lib = load_library()
    v = np.ascontiguousarray(vertices, np.float32).reshape(-1, 9)
    n = v.shape[0]
    g = None if geom_ids is None else np.ascontiguousarray(geom_ids, np.uint32)
    if g is not None and g.shape[0] != n:
        raise ValueError("geom_ids must have one entry per triangle")
    nb, tb = rt_bvh_buffer_bytes(n)
    # 16-byte aligned host buffers (records are viewed as float4)
    nodes = np.zeros(max(nb, 16) // 16, dtype=np.dtype((np.void, 16)))
    tris = np.zeros(max(tb, 16) // 16, dtype=np.dtype((np.void, 16)))
    info = rt_bvh_info()
    params = rt_build_params(int(max_leaf))
    _check(lib.rt_bvh_build_ex(v.ctypes.data if n else None, None if g is None else g.ctypes.data,
                               n, C.byref(params), nodes.ctypes.data if nb else None, nb,
                               tris.ctypes.data if tb else None, tb, C.byref(info)),
           "rt_bvh_build_ex")
    nodes_u8 = nodes.view(np.uint8)[: info.n_nodes * RT_NODE_BYTES]
    tris_u8 = tris.view(np.uint8)[: n * RT_TRI_BYTES]
    return nodes_u8, tris_u8, info


def rt_trace_workspace_bytes(scene: rt_scene, n_rays: int, flags: int = 0) -> int:
    lib = load_library()
    b = C.c_size_t()
    _check(lib.rt_trace_workspace_bytes(C.byref(scene), n_rays, flags, C.byref(b)),
           "rt_trace_workspace_bytes")
    return b.value


def rt_trace_closest(scene: rt_scene, rays_ptr: int, n_rays: int, kind: int, params,
                     flags: int, hits_ptr: int, counters_ptr: int | None, workspace_ptr: int | None,
                     workspace_bytes: int, stream: int | None):
    lib = load_library()
    _check(lib.rt_trace_closest(C.byref(scene), rays_ptr, n_rays, kind,
                                None if params is None else C.cast(C.pointer(params), C.c_void_p),
                                flags, hits_ptr, counters_ptr, workspace_ptr, workspace_bytes,
                                stream), "rt_trace_closest")


def rt_trace_closest_noalloc(scene: rt_scene, rays_ptr: int, n_rays: int, kind: int, params,
                             flags: int, hits_ptr: int, counters_ptr: int | None,
                             stream: int | None):
    lib = load_library()
    _check(lib.rt_trace_closest_noalloc(C.byref(scene), rays_ptr, n_rays, kind,
                                        None if params is None else
                                        C.cast(C.pointer(params), C.c_void_p),
                                        flags, hits_ptr, counters_ptr, stream),
           "rt_trace_closest_noalloc")


def rt_trace_any(scene: rt_scene, rays_ptr: int, n_rays: int, kind: int, params, flags: int,
                 occluder_ptr: int, counters_ptr: int | None, workspace_ptr: int | None,
                 workspace_bytes: int, stream: int | None):
    lib = load_library()
    _check(lib.rt_trace_any(C.byref(scene), rays_ptr, n_rays, kind,
                            None if params is None else C.cast(C.pointer(params), C.c_void_p),
                            flags, occluder_ptr, counters_ptr, workspace_ptr, workspace_bytes,
                            stream), "rt_trace_any")


def rt_batch_table_bytes(n_scenes: int) -> int:
    b = C.c_size_t()
    _check(load_library().rt_batch_table_bytes(n_scenes, C.byref(b)), "rt_batch_table_bytes")
    return b.value


def rt_batch_pack(entries, kind: int):
    """Packs rt_batch_entry structures into a host table.  Returns
    (table uint8 array, rt_batch_info)."""
    n = len(entries)
    arr = (rt_batch_entry * n)(*entries)
    nbytes = rt_batch_table_bytes(n)
    table = np.zeros((nbytes + 15) // 16, dtype=np.dtype((np.void, 16)))
    info = rt_batch_info()
    _check(load_library().rt_batch_pack(C.cast(arr, C.c_void_p), n, kind, table.ctypes.data,
                                        nbytes, C.byref(info)), "rt_batch_pack")
    return table.view(np.uint8)[:nbytes], info


def rt_trace_batch_workspace_bytes(info: rt_batch_info, flags: int = 0) -> int:
    b = C.c_size_t()
    _check(load_library().rt_trace_batch_workspace_bytes(C.byref(info), flags, C.byref(b)),
           "rt_trace_batch_workspace_bytes")
    return b.value


def rt_trace_batch(table_ptr: int, info: rt_batch_info, rays_ptr: int, kind: int, params,
                   flags: int, hits_ptr: int, counters_ptr: int | None, workspace_ptr: int | None,
                   workspace_bytes: int, stream: int | None):
    _check(load_library().rt_trace_batch(
        table_ptr, C.byref(info), rays_ptr, kind,
        None if params is None else C.cast(C.pointer(params), C.c_void_p), flags, hits_ptr,
        counters_ptr, workspace_ptr, workspace_bytes, stream), "rt_trace_batch")


def _instances(inst_blas, inst_m, world_lo, world_hi):
    n = len(inst_blas)
    arr = (rt_instance * max(1, n))()
    m = np.ascontiguousarray(inst_m, np.float32).reshape(-1, 12)
    lo = np.ascontiguousarray(world_lo, np.float32).reshape(-1, 3)
    hi = np.ascontiguousarray(world_hi, np.float32).reshape(-1, 3)
    for q in range(n):
        arr[q].blas = int(inst_blas[q])
        arr[q].object_from_world[:] = m[q].tolist()
        arr[q].world_lo[:] = lo[q].tolist()
        arr[q].world_hi[:] = hi[q].tolist()
    return arr, n


def rt_tlas_build(inst_blas, inst_m, world_lo, world_hi):
    """Host build of the top-level BVH; returns (nodes, tris, info) like rt_bvh_build."""
    arr, n = _instances(inst_blas, inst_m, world_lo, world_hi)
    nb, tb = rt_bvh_buffer_bytes(n)
    nodes = np.zeros(max(nb, 16) // 16, dtype=np.dtype((np.void, 16)))
    tris = np.zeros(max(tb, 16) // 16, dtype=np.dtype((np.void, 16)))
    info = rt_bvh_info()
    _check(load_library().rt_tlas_build(C.cast(arr, C.c_void_p), n,
                                        nodes.ctypes.data if nb else None, nb,
                                        tris.ctypes.data if tb else None, tb, C.byref(info)),
           "rt_tlas_build")
    return nodes.view(np.uint8)[: info.n_nodes * RT_NODE_BYTES], tris.view(np.uint8)[: n * RT_TRI_BYTES], info


def rt_instance_pack(blas_views, inst_blas, inst_m, world_lo, world_hi, texcoords=None):
    """Packs the instance table on the host; returns (table uint8, rt_instance_info).

    ``texcoords``: None, or one (device pointer or None, n_prims) pair per
    bottom-level scene, for the alpha mask."""
    lib = load_library()
    arr, n = _instances(inst_blas, inst_m, world_lo, world_hi)
    nb = len(blas_views)
    scenes = (rt_scene * max(1, nb))(*blas_views)
    tcs = None
    if texcoords is not None:
        if len(texcoords) != nb:
            raise ValueError("one texcoords entry per bottom-level scene")
        tcs = (rt_mesh_texcoords * max(1, nb))(
            *[rt_mesh_texcoords(p, int(m)) for p, m in texcoords])
    b = C.c_size_t()
    _check(lib.rt_instance_table_bytes(nb, n, C.byref(b)), "rt_instance_table_bytes")
    table = np.zeros((b.value + 15) // 16, dtype=np.dtype((np.void, 16)))
    info = rt_instance_info()
    _check(lib.rt_instance_pack(C.cast(scenes, C.c_void_p),
                                None if tcs is None else C.cast(tcs, C.c_void_p), nb,
                                C.cast(arr, C.c_void_p), n, table.ctypes.data, b.value,
                                C.byref(info)), "rt_instance_pack")
    return table.view(np.uint8)[: b.value], info


class InstancedScene:
    """Bottom-level scenes + instances: a device top-level BVH and table.

    For the alpha mask give every mesh its texture ids (``geom_ids``, one
    list entry per mesh, as in ``upload_scene``) and texture coordinates
    (``texcoords``, [n_tris, 3, 2] per mesh), and ``textures`` shared by all
    meshes ([n_tex, H, W] RGBA8 packed in uint32)."""

    def __init__(self, blas_vertices, inst_blas, inst_m, world_lo, world_hi, device="cuda", *,
                 geom_ids=None, texcoords=None, textures=None, max_leaf: int = 4):
        torch = _torch()
        nb = len(blas_vertices)
        gids = geom_ids if geom_ids is not None else [None] * nb
        tcs = texcoords if texcoords is not None else [None] * nb
        if len(gids) != nb or len(tcs) != nb:
            raise ValueError("geom_ids/texcoords need one entry per bottom-level scene")
        self.blas = [upload_scene(v, g, t, device=device, max_leaf=max_leaf)
                     for v, g, t in zip(blas_vertices, gids, tcs)]
        nodes, tris, self.tlas_info = rt_tlas_build(inst_blas, inst_m, world_lo, world_hi)
        self.tlas_nodes = torch.from_numpy(nodes.copy()).to(device) if nodes.size else None
        self.tlas_tris = torch.from_numpy(tris.copy()).to(device)
        mesh_tc = None
        if texcoords is not None:
            mesh_tc = [(b.texcoords.data_ptr() if b.texcoords is not None and b.texcoords.numel()
                        else None, 0 if b.texcoords is None else b.texcoords.numel() // 6)
                       for b in self.blas]
        table, self.info = rt_instance_pack([b.view for b in self.blas], inst_blas, inst_m,
                                            world_lo, world_hi, mesh_tc)
        self.max_blas_depth = int(self.info.max_blas_depth)
        self.table = torch.from_numpy(table.copy()).to(device)
        self.textures = None if textures is None else torch.from_numpy(
            np.ascontiguousarray(textures, np.uint32).view(np.int32)).to(device)

    @property
    def tlas(self) -> rt_scene:
        sc = rt_scene()
        sc.nodes = self.tlas_nodes.data_ptr() if self.tlas_nodes is not None else None
        sc.tris = self.tlas_tris.data_ptr() if self.tlas_tris.numel() else None
        sc.info = self.tlas_info
        return sc

    def _alpha_params(self, alpha_min: int) -> rt_alpha_params:
        if self.textures is None:
            raise ValueError("the alpha mask needs textures")
        p = rt_alpha_params()
        p.texcoords = None
        p.n_texcoord_prims = 0
        p.textures = self.textures.data_ptr()
        p.n_tex = int(self.textures.shape[0])
        p.height = int(self.textures.shape[1])
        p.width = int(self.textures.shape[2])
        p.alpha_min = int(alpha_min)
        return p

    def trace(self, rays, intersector="default", *, any_hit=False, count=False, checker_n=8,
              alpha_min=128, out=None, inst_ids=None, workspace=None, stream=None,
              image_width: int | None = None):
        """Returns (hits [N,4] float32 or occluders [N] int32, inst_ids [N] int32[,
        counters]).  ``stream``, ``image_width``: as for :func:`trace`."""
        with _on_stream(rays.device, stream) as s:
            return self._trace_on(rays, intersector, any_hit, count, checker_n, alpha_min, out,
                                  inst_ids, workspace, s, image_width)

    def _trace_on(self, rays, intersector, any_hit, count, checker_n, alpha_min, out, inst_ids,
                  workspace, s, image_width=None):
        torch = _torch()
        n = int(rays.shape[0])
        dev = rays.device
        if out is None:
            out = (torch.empty((n,), dtype=torch.int32, device=dev) if any_hit
                   else torch.empty((n, 4), dtype=torch.float32, device=dev))
        if inst_ids is None:
            inst_ids = torch.empty((n,), dtype=torch.int32, device=dev)
        counters = torch.empty((n, 4), dtype=torch.int32, device=dev) if count else None
        params = None
        if intersector == "procedural":
            params = rt_procedural_params()
            params.checker_n = int(checker_n)
        elif intersector == "alpha":
            params = self._alpha_params(alpha_min)
        elif intersector != "default":
            raise ValueError(f"unknown intersector {intersector!r}")
        flags = (RT_FLAG_COUNT if count else 0) | tile_flag(image_width)
        tl = self.tlas
        lib = load_library()
        b = C.c_size_t()
        _check(lib.rt_trace_instanced_workspace_bytes(C.byref(tl), C.byref(self.info), n, flags,
                                                      C.byref(b)), "rt_trace_instanced_workspace_bytes")
        ws = workspace or Workspace(dev)
        wptr, wbytes = ws.get(b.value)
        _check(lib.rt_trace_instanced(
            C.byref(tl), self.table.data_ptr(), C.byref(self.info), rays.data_ptr(), n,
            KINDS[intersector], None if params is None else C.cast(C.pointer(params), C.c_void_p),
            flags, int(bool(any_hit)), out.data_ptr(), inst_ids.data_ptr(),
            counters.data_ptr() if count else None, wptr, wbytes, s), "rt_trace_instanced")
        return (out, inst_ids, counters) if count else (out, inst_ids)


def rt_trace_multi(scene: rt_scene, rays_ptr: int, n_rays: int, kind: int, params, flags: int,
                   k: int, hits_ptr: int, n_hits_ptr: int, counters_ptr: int | None,
                   workspace_ptr: int | None, workspace_bytes: int, stream: int | None):
    lib = load_library()
    _check(lib.rt_trace_multi(C.byref(scene), rays_ptr, n_rays, kind,
                              None if params is None else C.cast(C.pointer(params), C.c_void_p),
                              flags, k, hits_ptr, n_hits_ptr, counters_ptr, workspace_ptr,
                              workspace_bytes, stream), "rt_trace_multi")


def rt_hit_backward(rays_ptr: int, hits_ptr: int, grad_tuv_ptr: int, n_rays: int,
                    vertices_ptr: int, n_vertices: int, faces_ptr: int, n_tris: int,
                    grad_vertices_ptr: int, grad_rays_ptr: int | None, stream: int | None):
    _check(load_library().rt_hit_backward(rays_ptr, hits_ptr, grad_tuv_ptr, n_rays, vertices_ptr,
                                          n_vertices, faces_ptr, n_tris, grad_vertices_ptr,
                                          grad_rays_ptr, stream), "rt_hit_backward")


def rt_launch_shapes():
    """[(block, lds_stack, chunk, queue), ...]; the first is the default."""
    lib = load_library()
    n = lib.rt_launch_shapes(None, None, None, None, 0)
    arr = [(C.c_uint32 * n)() for _ in range(4)]
    lib.rt_launch_shapes(*arr, n)
    return [tuple(int(a[i]) for a in arr) for i in range(n)]


def RT_FLAG_SHAPE(index: int) -> int:
    """The flags field that selects launch shape ``index`` of rt_launch_shapes()."""
    return (int(index) << RT_FLAG_SHAPE_SHIFT) & RT_FLAG_SHAPE_MASK


def shape_flag(shape) -> int:
    """Flags bits for a launch shape given as None (the default), an index into
    rt_launch_shapes(), or a (block, lds_stack, chunk, queue) tuple."""
    if shape is None:
        return 0
    if isinstance(shape, (int, np.integer)):
        return RT_FLAG_SHAPE(int(shape))
    shapes = rt_launch_shapes()
    key = tuple(int(x) for x in shape)
    if key not in shapes:
        raise RtxError(RT_ERR_UNSUPPORTED, "shape_flag", f"launch shape {key} not compiled in")
    return RT_FLAG_SHAPE(shapes.index(key))


def rt_status_string(status: int) -> str:
    return load_library().rt_status_string(status).decode()


def rt_last_error() -> str:
    return load_library().rt_last_error().decode()


# ----------------------------------------------------------------------------
# torch-side helpers
# ----------------------------------------------------------------------------
def _torch():
    import torch
    return torch


@dataclass
class Scene:
    """A BVH resident in device memory plus the optional alpha-mask data."""
    nodes: object            # torch uint8 tensor on the device (or None)
    tris: object             # torch uint8 tensor on the device
    info: rt_bvh_info
    texcoords: object = None  # torch float32 [n, 3, 2]
    textures: object = None   # torch int32 [n_tex, H, W] (RGBA8 bits)

    @property
    def view(self) -> rt_scene:
        sc = rt_scene()
        sc.nodes = self.nodes.data_ptr() if self.nodes is not None and self.nodes.numel() else None
        sc.tris = self.tris.data_ptr() if self.tris.numel() else None
        sc.info = self.info
        return sc

    def alpha_params(self, alpha_min: int = 128) -> rt_alpha_params:
        if self.texcoords is None or self.textures is None:
            raise ValueError("scene has no alpha-mask data")
        p = rt_alpha_params()
        p.texcoords = self.texcoords.data_ptr()
        p.textures = self.textures.data_ptr()
        p.n_texcoord_prims = int(self.texcoords.shape[0])
        p.n_tex, p.height, p.width = (int(s) for s in self.textures.shape)
        p.alpha_min = int(alpha_min)
        return p


def rt_bvh_compress(nodes: np.ndarray, info: rt_bvh_info):
    """64-byte nodes (from rt_bvh_build) -> 32-byte nodes with 8-bit child
    boxes.  Returns ``(nodes uint8, info)`` with ``info.layout = 1``."""
    n = int(info.n_nodes)
    src = np.ascontiguousarray(nodes, np.uint8)
    src16 = np.zeros(max(1, n * RT_NODE_BYTES // 16), dtype=np.dtype((np.void, 16)))
    src16.view(np.uint8)[: n * RT_NODE_BYTES] = src[: n * RT_NODE_BYTES]
    out = np.zeros(max(1, n * RT_NODE_BYTES_Q8 // 16), dtype=np.dtype((np.void, 16)))
    oinfo = rt_bvh_info()
    _check(load_library().rt_bvh_compress(src16.ctypes.data if n else None, C.byref(info),
                                           out.ctypes.data if n else None, n * RT_NODE_BYTES_Q8,
                                           C.byref(oinfo)), "rt_bvh_compress")
    return out.view(np.uint8)[: n * RT_NODE_BYTES_Q8], oinfo


def rt_bvh_pack(nodes: np.ndarray, info: rt_bvh_info):
    """64-byte nodes (from rt_bvh_build) -> 48-byte nodes carrying the child
    references in the low bytes of moved box words.  Returns ``(nodes uint8,
    info)`` with ``info.layout = 3``."""
    n = int(info.n_nodes)
    src = np.ascontiguousarray(nodes, np.uint8)
    src16 = np.zeros(max(1, n * RT_NODE_BYTES // 16), dtype=np.dtype((np.void, 16)))
    src16.view(np.uint8)[: n * RT_NODE_BYTES] = src[: n * RT_NODE_BYTES]
    out = np.zeros(max(1, n * RT_NODE_BYTES_F32P // 16), dtype=np.dtype((np.void, 16)))
    oinfo = rt_bvh_info()
    _check(load_library().rt_bvh_pack(src16.ctypes.data if n else None, C.byref(info),
                                       out.ctypes.data if n else None, n * RT_NODE_BYTES_F32P,
                                       C.byref(oinfo)), "rt_bvh_pack")
    return out.view(np.uint8)[: n * RT_NODE_BYTES_F32P], oinfo


def rt_bvh_refit_plan(nodes: np.ndarray, info: rt_bvh_info):
    """The refit plan of a built tree (64-byte nodes): ``(plan uint32
    [2 n_nodes + n_top], n_top)`` -- parent words, depths (bit 31: top node),
    the top nodes; ``(empty, 0)`` for a root leaf."""
    n = int(info.n_nodes)
    nt = C.c_uint32()
    if n == 0 or int(info.root_ref) >> 29:
        _check(load_library().rt_bvh_refit_plan(None, C.byref(info), None, 0, C.byref(nt)),
               "rt_bvh_refit_plan")
        return np.zeros(0, np.uint32), 0
    src = np.ascontiguousarray(nodes, np.uint8)
    src16 = np.zeros(n * RT_NODE_BYTES // 16, dtype=np.dtype((np.void, 16)))
    src16.view(np.uint8)[:] = src[: n * RT_NODE_BYTES]
    plan = np.zeros(3 * n, np.uint32)
    _check(load_library().rt_bvh_refit_plan(src16.ctypes.data, C.byref(info), plan.ctypes.data,
                                             plan.size, C.byref(nt)), "rt_bvh_refit_plan")
    return plan[: 2 * n + nt.value].copy(), int(nt.value)


def rt_bvh_widen(nodes: np.ndarray, info: rt_bvh_info):
    """64-byte binary nodes (from rt_bvh_build) -> 128-byte four-wide nodes.
    Returns ``(nodes uint8, info)`` with ``info.layout = 2``, ``info.n_nodes``
    the wide node count and ``info.max_depth`` the stack bound."""
    n = int(info.n_nodes)
    src = np.ascontiguousarray(nodes, np.uint8)
    src16 = np.zeros(max(1, n * RT_NODE_BYTES // 16), dtype=np.dtype((np.void, 16)))
    src16.view(np.uint8)[: n * RT_NODE_BYTES] = src[: n * RT_NODE_BYTES]
    out = np.zeros(max(1, n * RT_NODE_BYTES_WIDE4 // 16), dtype=np.dtype((np.void, 16)))
    oinfo = rt_bvh_info()
    _check(load_library().rt_bvh_widen(src16.ctypes.data if n else None, C.byref(info),
                                        out.ctypes.data if n else None, n * RT_NODE_BYTES_WIDE4,
                                        C.byref(oinfo)), "rt_bvh_widen")
    return out.view(np.uint8)[: int(oinfo.n_nodes) * RT_NODE_BYTES_WIDE4], oinfo


def upload_scene(vertices, geom_ids=None, texcoords=None, textures=None, device="cuda",
                 layout: str = "f32", max_leaf: int = 4) -> Scene:
    """Builds the BVH on the host (rt_bvh_build_ex with leaves of at most
    ``max_leaf`` triangles, then rt_bvh_compress for ``layout="q8"``,
    rt_bvh_pack for ``layout="f32p"`` or rt_bvh_widen for ``layout="wide4"``)
    and copies it to ``device``."""
    torch = _torch()
    if layout not in LAYOUTS:
        raise ValueError(f"unknown layout {layout!r}")
    nodes, tris, info = rt_bvh_build(vertices, geom_ids, max_leaf)
    if layout == "q8":
        nodes, info = rt_bvh_compress(nodes, info)
    elif layout == "f32p":
        nodes, info = rt_bvh_pack(nodes, info)
    elif layout == "wide4":
        nodes, info = rt_bvh_widen(nodes, info)
    dn = torch.from_numpy(nodes.copy()).to(device) if nodes.size else None
    dt = torch.from_numpy(tris.copy()).to(device)
    tc = None if texcoords is None else torch.from_numpy(
        np.ascontiguousarray(texcoords, np.float32)).to(device)
    tx = None if textures is None else torch.from_numpy(
        np.ascontiguousarray(textures, np.uint32).view(np.int32)).to(device)
    return Scene(dn, dt, info, tc, tx)


class RefitScene:
    """A scene built once from an indexed mesh whose vertices then move:
    ``update(vertices)`` refits it on the device (rt_bvh_refit, the topology
    kept) instead of rebuilding it on the host.  ``scene`` is the traceable
    Scene (64-byte nodes); ``faces`` stays on the device."""

    def __init__(self, vertices, faces, geom_ids=None, texcoords=None, textures=None,
                 device="cuda", max_leaf: int = 4):
        torch = _torch()
        v = np.ascontiguousarray(vertices, np.float32).reshape(-1, 3)
        f = np.ascontiguousarray(faces, np.int64).reshape(-1, 3)
        if f.size and (f.min() < 0 or f.max() >= v.shape[0]):
            raise ValueError("faces must index the vertices")
        nodes, tris, info = rt_bvh_build(v[f], geom_ids, max_leaf)
        plan, self.n_top = rt_bvh_refit_plan(nodes, info)
        dn = torch.from_numpy(nodes.copy()).to(device) if nodes.size else None
        dt = torch.from_numpy(tris.copy()).to(device)
        tc = None if texcoords is None else torch.from_numpy(
            np.ascontiguousarray(texcoords, np.float32)).to(device)
        tx = None if textures is None else torch.from_numpy(
            np.ascontiguousarray(textures, np.uint32).view(np.int32)).to(device)
        self.scene = Scene(dn, dt, info, tc, tx)
        self.plan = torch.from_numpy(plan.view(np.int32)).to(device) if plan.size else None
        self.faces = torch.from_numpy(f.astype(np.int32)).to(device)
        self.n_vertices = v.shape[0]
        self.root_box = torch.empty(6, dtype=torch.float32, device=device)

    def update(self, vertices, stream=None):
        """Refits to ``vertices`` (device float32 [n_vertices, 3]) and sets the
        scene's root box (one 24-byte copy to the host, which waits for the
        refit)."""
        torch = _torch()
        if (vertices.dtype != torch.float32 or vertices.dim() != 2 or vertices.shape[1] != 3
                or not vertices.is_contiguous() or vertices.shape[0] != self.n_vertices):
            raise ValueError(f"vertices must be a contiguous float32 [{self.n_vertices}, 3] tensor")
        if vertices.device != self.faces.device:
            raise ValueError("vertices must be on the scene's device")
        with _on_stream(vertices.device, stream) as s:
            sc = self.scene.view
            _check(load_library().rt_bvh_refit(
                C.byref(sc), None if self.plan is None else self.plan.data_ptr(), self.n_top,
                vertices.data_ptr(), self.n_vertices, self.faces.data_ptr(),
                self.root_box.data_ptr(), s),
                "rt_bvh_refit")
            if int(self.scene.info.n_tris) > 0:
                box = self.root_box.cpu().numpy()
                for a in range(3):
                    self.scene.info.root_lo[a] = float(box[a])
                    self.scene.info.root_hi[a] = float(box[3 + a])
        return self.scene


def _params(scene: Scene, intersector: str, alpha_min: int, checker_n: int):
    if intersector not in KINDS:
        raise ValueError(f"unknown intersector {intersector!r}")
    if intersector == "alpha":
        return scene.alpha_params(alpha_min)
    if intersector == "procedural":
        p = rt_procedural_params()
        p.checker_n = int(checker_n)
        return p
    return None


class _on_stream:
    """Context for one trace call: yields the raw stream to launch on.  When
    the caller names a stream other than torch's current one, torch's current
    stream is switched to it for the call, so that the outputs and any
    temporary workspace allocated here belong to the stream the kernel runs
    on (the caching allocator then never hands their memory to other work
    while the kernel may still use it)."""

    def __init__(self, device, stream):
        self.device, self.stream, self.ctx = device, stream, None

    def __enter__(self):
        torch = _torch()
        cur = torch.cuda.current_stream(self.device)
        if self.stream is None or int(self.stream) == int(cur.cuda_stream):
            return cur.cuda_stream
        ext = torch.cuda.ExternalStream(int(self.stream), device=self.device)
        self.ctx = torch.cuda.stream(ext)
        self.ctx.__enter__()
        return int(self.stream)

    def __exit__(self, *exc):
        if self.ctx is not None:
            self.ctx.__exit__(*exc)
        return False


class Workspace:
    """Caller-owned device workspace reused across trace calls."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = None

    def get(self, nbytes: int):
        torch = _torch()
        if nbytes == 0:
            return None, 0
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self.buf.data_ptr(), int(self.buf.numel())


def tile_flag(image_width: int | None) -> int:
    """Flag bits of the tiled schedule for rays forming an image of this
    width in scanline order (None or 0: index order)."""
    if not image_width:
        return 0
    if image_width % 8 or not 0 < image_width <= 8 * 0xFFF:
        raise ValueError("tiled schedule: image width must be a multiple of 8, at most 32760")
    return (image_width // 8) << RT_FLAG_TILE_SHIFT


def waves_flag(waves_per_simd: int | None) -> int:
    """Flag bits capping a queue launch's persistent grid at this many waves
    per SIMD (1..15; None or 0: the library default, 7)."""
    if not waves_per_simd:
        return 0
    if not 1 <= int(waves_per_simd) <= 15:
        raise ValueError("waves per SIMD must be within 1..15")
    return int(waves_per_simd) << RT_FLAG_WAVES_SHIFT


def trace(scene: Scene, rays, intersector: str = "default", *, query: str = "closest",
          count: bool = False, alpha_min: int = 128, checker_n: int = 8, k: int = 4, out=None,
          counters=None, workspace: Workspace | None = None, stream=None, shape=None,
          image_width: int | None = None, longest_first: bool = False,
          waves_per_simd: int | None = None):
    """Traces device rays ``float32 [N, 8]``.

    closest: returns ``hits float32 [N, 4]`` = (t, prim_id bits, u, v); view
    column 1 as int32/uint32 for prim_id.  any: returns ``int32 [N]``
    occluders (-1 = none).  multi: returns ``(hits float32 [N, k, 4], n_hits
    int32 [N])``.  With ``count`` also returns ``int32 [N, 4]`` counters (box
    tests, triangle tests, candidates, accepted).  ``shape``: launch shape of
    this call (see :func:`shape_flag`; None = the library's default).
    ``stream``: a raw hipStream_t to launch on instead of torch's current
    stream; the tensors allocated here are then allocated on that stream.
    ``image_width``: the rays are an image of this width in scanline order;
    lanes then take them in 8 x 8 tiles (same results, see
    ``RT_FLAG_TILE_WIDTH``).  ``longest_first``: hand out the chunks of rays
    that cross the most scene first (same results, see
    ``RT_FLAG_LONGEST_FIRST``).  ``waves_per_simd``: most resident waves per
    SIMD of a queue shape's persistent grid, which sets the rays per lane
    (same results, see ``RT_FLAG_WAVES_PER_SIMD``; None: the default, 7)."""
    torch = _torch()
    if rays.dtype != torch.float32 or rays.dim() != 2 or rays.shape[1] != 8 or not rays.is_contiguous():
        raise ValueError("rays must be a contiguous float32 [N, 8] tensor")
    with _on_stream(rays.device, stream) as s:
        return _trace_on(scene, rays, intersector, query, count, alpha_min, checker_n, k, out,
                         counters, workspace, s, shape, image_width, longest_first,
                         waves_per_simd)


def _trace_on(scene, rays, intersector, query, count, alpha_min, checker_n, k, out, counters,
              workspace, s, shape, image_width=None, longest_first=False, waves_per_simd=None):
    torch = _torch()
    n = int(rays.shape[0])
    dev = rays.device
    params = _params(scene, intersector, alpha_min, checker_n)
    flags = ((RT_FLAG_COUNT if count else 0) | shape_flag(shape) | tile_flag(image_width)
             | (RT_FLAG_LONGEST_FIRST if longest_first else 0) | waves_flag(waves_per_simd))
    sc = scene.view
    if query == "closest":
        if out is None:
            out = torch.empty((n, 4), dtype=torch.float32, device=dev)
    elif query == "any":
        if out is None:
            out = torch.empty((n,), dtype=torch.int32, device=dev)
    elif query == "multi":
        if out is None:
            out = torch.empty((n, k, 4), dtype=torch.float32, device=dev)
        n_hits = torch.empty((n,), dtype=torch.int32, device=dev)
    else:
        raise ValueError("query must be 'closest', 'any' or 'multi'")
    if count and counters is None:
        counters = torch.empty((n, 4), dtype=torch.int32, device=dev)
    ws = workspace or Workspace(dev)
    wptr, wbytes = ws.get(rt_trace_workspace_bytes(sc, n, flags))
    cptr = counters.data_ptr() if count else None
    if query == "closest":
        rt_trace_closest(sc, rays.data_ptr(), n, KINDS[intersector], params, flags,
                         out.data_ptr(), cptr, wptr, wbytes, s)
    elif query == "any":
        rt_trace_any(sc, rays.data_ptr(), n, KINDS[intersector], params, flags,
                     out.data_ptr(), cptr, wptr, wbytes, s)
    else:
        rt_trace_multi(sc, rays.data_ptr(), n, KINDS[intersector], params, flags, k,
                       out.data_ptr(), n_hits.data_ptr(), cptr, wptr, wbytes, s)
        out = (out, n_hits)
    return (out, counters) if count else out


class Batch:
    """Scenes with their ray counts, packed into a device scene table
    (rt_batch_pack + one host-to-device copy made here, by torch)."""

    def __init__(self, scenes, n_rays, intersector: str = "default", alpha_min=128,
                 device="cuda"):
        torch = _torch()
        self.scenes = list(scenes)
        self.kind = KINDS[intersector]
        self.intersector = intersector
        entries = []
        mins = ([int(alpha_min)] * len(self.scenes) if np.ndim(alpha_min) == 0
                else [int(a) for a in alpha_min])   # one threshold, or one per scene
        for sc, n, amin in zip(self.scenes, n_rays, mins):
            e = rt_batch_entry()
            e.scene = sc.view
            e.n_rays = int(n)
            if intersector == "alpha":
                e.alpha = sc.alpha_params(amin)
            entries.append(e)
        table, self.info = rt_batch_pack(entries, self.kind)
        self.table = torch.from_numpy(table.copy()).to(device)
        self.offsets = np.concatenate([[0], np.cumsum(np.asarray(n_rays, np.int64))])

    def trace(self, rays, *, count=False, checker_n: int = 8, out=None, counters=None,
              workspace: Workspace | None = None, stream=None, shape=None,
              waves_per_simd: int | None = None):
        """Closest hits of all rays (scene order) in one launch (``shape``,
        ``stream``, ``waves_per_simd``: as for :func:`trace`)."""
        torch = _torch()
        n = int(self.info.n_rays)
        if rays.shape != (n, 8) or rays.dtype != torch.float32 or not rays.is_contiguous():
            raise ValueError(f"rays must be a contiguous float32 [{n}, 8] tensor")
        with _on_stream(rays.device, stream) as s:
            return self._trace_on(rays, count, checker_n, out, counters, workspace, s, shape,
                                  waves_per_simd)

    def _trace_on(self, rays, count, checker_n, out, counters, workspace, s, shape,
                  waves_per_simd=None):
        torch = _torch()
        n = int(self.info.n_rays)
        dev = rays.device
        if out is None:
            out = torch.empty((n, 4), dtype=torch.float32, device=dev)
        flags = (RT_FLAG_COUNT if count else 0) | shape_flag(shape) | waves_flag(waves_per_simd)
        if count and counters is None:
            counters = torch.empty((n, 4), dtype=torch.int32, device=dev)
        params = None
        if self.intersector == "procedural":
            params = rt_procedural_params()
            params.checker_n = int(checker_n)
        ws = workspace or Workspace(dev)
        wptr, wbytes = ws.get(rt_trace_batch_workspace_bytes(self.info, flags))
        rt_trace_batch(self.table.data_ptr(), self.info, rays.data_ptr(), self.kind, params, flags,
                       out.data_ptr(), counters.data_ptr() if count else None, wptr, wbytes, s)
        return (out, counters) if count else out
