"""CPU oracle for custom-intersector ray traversal (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the product library never does.

Oracle A (:func:`brute`): float64 brute force over every triangle -- the plain
definition of the closest-hit / any-hit queries of Section 3.1, with the
alpha-mask and procedural intersectors of Section 4 evaluated in float64.

Oracle B (:func:`build_bvh`, :func:`traverse`): its own binned-SAH BVH and a
float32 while-while traversal (Algorithm 1) that counts ray/box and
ray/triangle tests the way the heat-map intersector of Section 4 does; with
``layout="q8"`` the inner nodes' child boxes are the 8-bit quantized boxes of
the 32-byte node layout (:func:`quantize`), with ``layout="f32p"`` the stored
boxes of the 48-byte packed-reference layout (:func:`pack`); the paper covers
neither.

The C source is ``rt_oracle.c``; :func:`build` compiles it with gcc.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rt_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

KINDS = {"default": 0, "alpha": 1, "procedural": 2}
MISS = 0xFFFFFFFF

E_NEAR_TIE = 1
E_NEAR_EDGE = 2
E_NEAR_FILTER = 4

NODE_DTYPE = np.dtype([("lo", "<f4", 3), ("hi", "<f4", 3), ("left", "<u4"), ("right", "<u4"),
                       ("first", "<u4"), ("count", "<u4"), ("depth", "<u4")])


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-pthread", "-Wall", "-Wextra", "-Wno-unused-parameter",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Isect(C.Structure):
    _fields_ = [("texcoords", C.c_void_p), ("textures", C.c_void_p), ("n_tex", C.c_uint32),
                ("width", C.c_uint32), ("height", C.c_uint32), ("alpha_min", C.c_uint32),
                ("checker_n", C.c_uint32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        lib.orc_brute.argtypes = [P, P, C.c_uint32, P, P, C.c_uint32, C.c_int, P, C.c_int,
                                  P, P, P, P, P, P, P, P, C.c_int]
        lib.orc_brute.restype = C.c_int
        lib.orc_build.argtypes = [P, C.c_uint32, P, P, P, P]
        lib.orc_build.restype = C.c_int
        lib.orc_build_leaf.argtypes = [P, C.c_uint32, C.c_uint32, P, P, P, P]
        lib.orc_build_leaf.restype = C.c_int
        lib.orc_traverse.argtypes = [P, P, C.c_uint32, P, P, C.c_uint32, P, C.c_uint32, C.c_int,
                                     P, C.c_int, C.c_uint32, P, P, P, P, P, P, C.c_int]
        lib.orc_brute_multi.argtypes = [P, P, C.c_uint32, P, C.c_uint32, C.c_int, P, C.c_uint32,
                                        P, P, P, P, P, P, C.c_int]
        lib.orc_brute_multi.restype = C.c_int
        lib.orc_traverse.restype = C.c_int
        lib.orc_traverse_layout.argtypes = [P, P, C.c_uint32, P, P, C.c_uint32, P, P, C.c_uint32,
                                            C.c_int, P, C.c_int, C.c_uint32, P, P, P, P, P, P,
                                            C.c_int]
        lib.orc_traverse_layout.restype = C.c_int
        lib.orc_traverse_wide.argtypes = [P, P, C.c_uint32, P, P, C.c_uint32, P, P, C.c_uint32,
                                          C.c_int, P, C.c_int, C.c_uint32, P, P, P, P, P, P,
                                          C.c_int]
        lib.orc_traverse_wide.restype = C.c_int
        lib.orc_widen.argtypes = [P, C.c_uint32, P, P, P, P]
        lib.orc_widen.restype = C.c_int
        lib.orc_quantize.argtypes = [P, C.c_uint32, P, P, P]
        lib.orc_quantize.restype = C.c_int
        lib.orc_refit.argtypes = [P, C.c_uint32, P, C.c_uint32, P, C.c_uint32, P]
        lib.orc_refit.restype = C.c_int
        lib.orc_pack.argtypes = [P, C.c_uint32, P, P]
        lib.orc_pack.restype = C.c_int
        lib.orc_move_word.argtypes = [C.c_float, C.c_uint32, C.c_int, C.POINTER(C.c_float)]
        lib.orc_move_word.restype = C.c_int
        lib.orc_node_size.restype = C.c_uint32
        lib.orc_fixed_hit64.argtypes = [P, P, P, P, C.c_uint32, P]
        lib.orc_fixed_hit64.restype = C.c_int
        lib.orc_hit_grad64.argtypes = [P, C.c_uint32, P, P, P, P, C.c_uint32, P, P]
        lib.orc_hit_grad64.restype = C.c_int
        lib.orc_brute_instanced.argtypes = [P, C.c_uint32, P, C.c_uint32, P, C.c_uint32, C.c_int, P,
                                            P, P, P, P, P, P, P, P]
        lib.orc_brute_instanced.restype = C.c_int
        lib.orc_traverse_instanced.argtypes = [P, C.c_uint32, P, C.c_uint32, P, P, P, C.c_uint32,
                                               C.c_int, P, C.c_int, P, P, P, P, P, P]
        lib.orc_traverse_instanced.restype = C.c_int
        assert lib.orc_node_size() == NODE_DTYPE.itemsize
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _threads(n):
    if n is not None:
        return int(n)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def _isect(texcoords, textures, alpha_min, checker_n):
    is_ = _Isect()
    keep = []
    if texcoords is not None:
        tc = np.ascontiguousarray(texcoords, np.float32)
        keep.append(tc)
        is_.texcoords = tc.ctypes.data
    if textures is not None:
        tx = np.ascontiguousarray(textures, np.uint32)
        keep.append(tx)
        is_.textures = tx.ctypes.data
        is_.n_tex, is_.height, is_.width = (int(s) for s in tx.shape)
    is_.alpha_min = int(alpha_min)
    is_.checker_n = int(checker_n)
    return is_, keep


def _check_kind(kind, geom_ids, texcoords, textures, n_tris):
    if kind not in KINDS:
        raise ValueError(f"unknown intersector {kind!r}")
    if kind == "alpha":
        if texcoords is None or textures is None:
            raise ValueError("alpha intersector needs texcoords and textures")
        if np.asarray(texcoords).shape[0] < n_tris:
            raise ValueError("texcoords must cover every triangle")
        if geom_ids is not None and n_tris and int(np.max(geom_ids)) >= np.asarray(textures).shape[0]:
            raise ValueError("geom_id out of range of the texture array")


def brute(vertices, rays, kind="default", *, geom_ids=None, texcoords=None, textures=None,
          alpha_min=128, checker_n=8, any_hit=False, ray_index=None, threads=None):
    """Oracle A.  Returns a dict with float64 ``t, u, v, t2, bound_uv, bound_t``,
    uint32 ``prim`` (``MISS`` for none) and uint8 exception ``flags``; entries
    follow ``ray_index`` when given."""
    lib = _load()
    verts = np.ascontiguousarray(vertices, np.float32).reshape(-1, 9)
    r = np.ascontiguousarray(rays, np.float32).reshape(-1, 8)
    n = verts.shape[0]
    _check_kind(kind, geom_ids, texcoords, textures, n)
    g = None if geom_ids is None else np.ascontiguousarray(geom_ids, np.uint32)
    idx = None if ray_index is None else np.ascontiguousarray(ray_index, np.int64)
    m = r.shape[0] if idx is None else idx.shape[0]
    out = {k: np.empty(m, np.float64) for k in ("t", "u", "v", "t2", "bound_uv", "bound_t")}
    out["prim"] = np.empty(m, np.uint32)
    out["flags"] = np.empty(m, np.uint8)
    is_, keep = _isect(texcoords, textures, alpha_min, checker_n)
    rc = lib.orc_brute(_ptr(verts), _ptr(g), n, _ptr(r), _ptr(idx), m, KINDS[kind],
                       C.byref(is_), int(bool(any_hit)), _ptr(out["t"]), _ptr(out["prim"]),
                       _ptr(out["u"]), _ptr(out["v"]), _ptr(out["t2"]), _ptr(out["flags"]),
                       _ptr(out["bound_uv"]), _ptr(out["bound_t"]), _threads(threads))
    if rc != 0:
        raise RuntimeError(f"orc_brute failed ({rc})")
    del keep
    return out


@dataclass
class OracleBVH:
    nodes: np.ndarray    # NODE_DTYPE, preorder, node 0 = root
    perm: np.ndarray     # uint32, leaf order -> input triangle index
    max_depth: int
    qbox: np.ndarray | None = field(default=None, repr=False)  # quantize()'s boxes, once computed
    wide: dict | None = field(default=None, repr=False)        # widen()'s layout, once computed
    pbox: np.ndarray | None = field(default=None, repr=False)  # pack()'s boxes, once computed

    @property
    def n_nodes(self) -> int:
        return int(self.nodes.shape[0])


def build_bvh(vertices, max_leaf: int = 4) -> OracleBVH:
    """Oracle B's own BVH build (binned SAH, leaves of at most ``max_leaf``
    triangles, 1..7)."""
    lib = _load()
    verts = np.ascontiguousarray(vertices, np.float32).reshape(-1, 9)
    n = verts.shape[0]
    nodes = np.zeros(max(1, 2 * n), NODE_DTYPE)
    perm = np.zeros(max(1, n), np.uint32)
    nn = C.c_uint32()
    md = C.c_uint32()
    rc = lib.orc_build_leaf(_ptr(verts), n, int(max_leaf), _ptr(nodes), _ptr(perm), C.byref(nn),
                            C.byref(md))
    if rc == -2:
        raise ValueError("max_leaf must be within 1..7")
    if rc != 0:
        raise MemoryError("orc_build failed")
    return OracleBVH(nodes[: nn.value].copy(), perm[:n].copy(), int(md.value))


def refit(bvh: OracleBVH, vertices, faces) -> OracleBVH:
    """The same tree with every box recomputed from an indexed mesh
    (``vertices [nv, 3]`` float32, ``faces [n, 3]`` by input triangle index):
    boxes grow from (+inf, -inf) by strict comparisons, a triangle's over its
    vertices 0, 1, 2, a leaf's over its triangles in leaf order, an inner
    node's over its first child's box then its second's; an index >= nv reads
    NaN.  Returns a new OracleBVH (the input is unchanged)."""
    lib = _load()
    v = np.ascontiguousarray(vertices, np.float32).reshape(-1, 3)
    f = np.ascontiguousarray(faces, np.uint32).reshape(-1, 3)
    nodes = bvh.nodes.copy()
    rc = lib.orc_refit(_ptr(nodes), bvh.n_nodes, _ptr(bvh.perm), int(bvh.perm.size), _ptr(v),
                       v.shape[0], _ptr(f))
    if rc != 0:
        raise ValueError("orc_refit: a leaf references a triangle past the mesh")
    return OracleBVH(nodes, bvh.perm.copy(), bvh.max_depth)


def quantize(bvh: OracleBVH) -> dict:
    """The 32-byte node layout of every inner node of an oracle BVH:
    ``frames [n_nodes, 3]`` uint32 (origin bits | scale exponent), ``q
    [n_nodes, 12]`` uint8 (qlo0.xyz, qhi0.xyz, qlo1.xyz, qhi1.xyz) and the
    decoded child boxes ``qbox [n_nodes, 12]`` float32 (lo0, hi0, lo1, hi1);
    leaf entries are zero."""
    lib = _load()
    n = bvh.n_nodes
    frames = np.zeros((n, 3), np.uint32)
    q = np.zeros((n, 12), np.uint8)
    qbox = np.zeros((n, 12), np.float32)
    if lib.orc_quantize(_ptr(bvh.nodes), n, _ptr(frames), _ptr(q), _ptr(qbox)) != 0:
        raise ValueError("orc_quantize: a box has no valid scale (non-finite coordinates)")
    return {"frames": frames, "q": q, "qbox": qbox}


def pack(bvh: OracleBVH) -> dict:
    """The packed-reference (48-byte) layout of every inner node of an oracle
    BVH: ``box [n_nodes, 12]`` float32, the stored child boxes (lo0, hi0,
    lo1, hi1) with each child's reference in the low bytes of its lo.x, lo.y,
    lo.z, hi.x, and ``refs [n_nodes, 2]`` uint32, the canonical child
    references (inner-node preorder index, or count << 29 | first); leaf
    entries are zero."""
    lib = _load()
    n = bvh.n_nodes
    box = np.zeros((n, 12), np.float32)
    refs = np.zeros((n, 2), np.uint32)
    if bvh.perm.size == 0:  # no triangles: the node array is a placeholder root
        return {"box": box, "refs": refs}
    rc = lib.orc_pack(_ptr(bvh.nodes), n, _ptr(box), _ptr(refs))
    if rc == -1:
        raise ValueError("orc_pack: a box bound cannot move without reaching an infinity")
    if rc != 0:
        raise MemoryError("orc_pack failed")
    return {"box": box, "refs": refs}


def move_word(x, byte: int, lower: bool):
    """The packed layout's move of one box word: the float32 nearest to ``x``
    outward (down if ``lower``) whose bit pattern's low byte is ``byte``, or
    None if the walk reaches an infinity."""
    out = C.c_float()
    if _load().orc_move_word(C.c_float(np.float32(x)), int(byte), int(bool(lower)),
                             C.byref(out)) != 0:
        return None
    return np.float32(out.value)


WIDE_DTYPE = np.dtype([("n", "<u4"), ("child", "<u4", 4)])
WIDE_STACK = 128  # entries of oracle B's traversal stack


def widen(bvh: OracleBVH) -> dict:
    """The four-wide layout of an oracle BVH: ``wide`` (one WIDE_DTYPE entry
    per binary node: child count and binary child indices of the wide node it
    heads, n = 0 for the others), ``order`` (the heads of the wide nodes in
    depth-first preorder), and ``stack_bound`` (the largest sum of k - 1 over
    the wide nodes of a root-to-leaf path)."""
    lib = _load()
    n = bvh.n_nodes
    wide = np.zeros(max(1, n), WIDE_DTYPE)
    order = np.zeros(max(1, n), np.uint32)
    nw, sb = C.c_uint32(), C.c_uint32()
    if lib.orc_widen(_ptr(bvh.nodes), n, _ptr(wide), _ptr(order), C.byref(nw), C.byref(sb)) != 0:
        raise RuntimeError("orc_widen failed")
    return {"wide": wide[:n], "order": order[: nw.value].copy(), "stack_bound": int(sb.value)}


def traverse(vertices, bvh: OracleBVH, rays, kind="default", *, geom_ids=None, texcoords=None,
             textures=None, alpha_min=128, checker_n=8, any_hit=False, count=True, multi_k=0,
             layout="f32", threads=None):
    """Oracle B traversal.  Returns float32 ``t, u, v``, uint32 ``prim`` and,
    with ``count``, uint32 ``counters [N, 4]`` = (box tests, triangle tests,
    candidates handed to the intersector, accepted candidates).  With
    ``multi_k > 0`` (multi-hit) ``t, u, v, prim`` are ``[N, multi_k]`` (nearest
    first, padded with misses) and ``n_hits [N]`` counts the kept hits.
    ``layout``: "f32" (float32 child boxes), "q8" (the 32-byte layout's
    quantized child boxes), "f32p" (the 48-byte layout's stored child boxes)
    or "wide4" (the four-wide layout of the same BVH)."""
    lib = _load()
    verts = np.ascontiguousarray(vertices, np.float32).reshape(-1, 9)
    r = np.ascontiguousarray(rays, np.float32).reshape(-1, 8)
    n = verts.shape[0]
    _check_kind(kind, geom_ids, texcoords, textures, n)
    g = None if geom_ids is None else np.ascontiguousarray(geom_ids, np.uint32)
    m = r.shape[0]
    shape = (m, multi_k) if multi_k else (m,)
    out = {k: np.empty(shape, np.float32) for k in ("t", "u", "v")}
    out["prim"] = np.empty(shape, np.uint32)
    nh = np.empty(m, np.uint32) if multi_k else None
    cnt = np.empty((m, 4), np.uint32) if count else None
    is_, keep = _isect(texcoords, textures, alpha_min, checker_n)
    if layout not in ("f32", "q8", "f32p", "wide4"):
        raise ValueError(f"unknown layout {layout!r}")
    qbox = None
    if layout == "q8":
        if bvh.qbox is None:
            bvh.qbox = quantize(bvh)["qbox"]
        qbox = bvh.qbox
    if layout == "f32p":
        if bvh.pbox is None:
            bvh.pbox = pack(bvh)["box"]
        qbox = bvh.pbox
    if layout == "wide4":
        if bvh.wide is None:
            bvh.wide = widen(bvh)
        if bvh.wide["stack_bound"] > WIDE_STACK:
            raise ValueError("four-wide stack bound exceeds the oracle's stack")
        rc = lib.orc_traverse_wide(_ptr(verts), _ptr(g), n, _ptr(bvh.nodes), _ptr(bvh.perm),
                                   bvh.n_nodes, _ptr(bvh.wide["wide"]), _ptr(r), m, KINDS[kind],
                                   C.byref(is_), int(bool(any_hit)), int(multi_k), _ptr(out["t"]),
                                   _ptr(out["prim"]), _ptr(out["u"]), _ptr(out["v"]), _ptr(nh),
                                   _ptr(cnt), _threads(threads))
    else:
        rc = lib.orc_traverse_layout(_ptr(verts), _ptr(g), n, _ptr(bvh.nodes), _ptr(bvh.perm),
                                     bvh.n_nodes, _ptr(qbox), _ptr(r), m, KINDS[kind],
                                     C.byref(is_), int(bool(any_hit)), int(multi_k),
                                     _ptr(out["t"]), _ptr(out["prim"]), _ptr(out["u"]),
                                     _ptr(out["v"]), _ptr(nh), _ptr(cnt), _threads(threads))
    if rc != 0:
        raise RuntimeError(f"orc_traverse failed ({rc})")
    if count:
        out["counters"] = cnt
    if multi_k:
        out["n_hits"] = nh
    del keep
    return out


def brute_multi(vertices, rays, k, kind="default", *, geom_ids=None, texcoords=None,
                textures=None, alpha_min=128, checker_n=8):
    """Oracle A for the multi-hit query: the k nearest accepted hits of every
    ray in float64 ([N, k], ties by input index, padded with misses), their
    number ``n_hits`` and exception ``flags``."""
    lib = _load()
    verts = np.ascontiguousarray(vertices, np.float32).reshape(-1, 9)
    r = np.ascontiguousarray(rays, np.float32).reshape(-1, 8)
    n = verts.shape[0]
    _check_kind(kind, geom_ids, texcoords, textures, n)
    g = None if geom_ids is None else np.ascontiguousarray(geom_ids, np.uint32)
    m = r.shape[0]
    out = {kk: np.empty((m, k), np.float64) for kk in ("t", "u", "v")}
    out["prim"] = np.empty((m, k), np.uint32)
    out["n_hits"] = np.empty(m, np.uint32)
    out["flags"] = np.empty(m, np.uint8)
    is_, keep = _isect(texcoords, textures, alpha_min, checker_n)
    rc = lib.orc_brute_multi(_ptr(verts), _ptr(g), n, _ptr(r), m, KINDS[kind], C.byref(is_), k,
                             _ptr(out["t"]), _ptr(out["prim"]), _ptr(out["u"]), _ptr(out["v"]),
                             _ptr(out["n_hits"]), _ptr(out["flags"]), 1)
    if rc != 0:
        raise RuntimeError(f"orc_brute_multi failed ({rc})")
    del keep
    return out


# ----------------------------------------------------------------------------
# gradient of the accepted hit
# ----------------------------------------------------------------------------
def fixed_hit64(vertices64, faces, rays, prims):
    """float64 (t, u, v) of each ray against its fixed triangle (NaN for
    misses); ``vertices64`` float64 [nv, 3], ``faces`` uint32 [n, 3]."""
    lib = _load()
    v = np.ascontiguousarray(vertices64, np.float64)
    f = np.ascontiguousarray(faces, np.uint32)
    r = np.ascontiguousarray(rays, np.float32).reshape(-1, 8)
    p = np.ascontiguousarray(prims, np.uint32)
    out = np.empty((r.shape[0], 3), np.float64)
    lib.orc_fixed_hit64(_ptr(v), _ptr(f), _ptr(r), _ptr(p), r.shape[0], _ptr(out))
    return out


def hit_grad64(vertices64, faces, rays, prims, grad_tuv):
    """float64 closed-form gradient of sum(grad_tuv * (t, u, v)) with the hit
    prims fixed.  Returns (grad_vertices [nv, 3], grad_rays [N, 6])."""
    lib = _load()
    v = np.ascontiguousarray(vertices64, np.float64)
    f = np.ascontiguousarray(faces, np.uint32)
    r = np.ascontiguousarray(rays, np.float32).reshape(-1, 8)
    p = np.ascontiguousarray(prims, np.uint32)
    g = np.ascontiguousarray(grad_tuv, np.float64)
    gv = np.zeros_like(v)
    gr = np.empty((r.shape[0], 6), np.float64)
    rc = lib.orc_hit_grad64(_ptr(v), v.shape[0], _ptr(f), _ptr(r), _ptr(p), _ptr(g), r.shape[0],
                            _ptr(gv), _ptr(gr))
    if rc != 0:
        raise ValueError("face index out of range")
    return gv, gr


# ----------------------------------------------------------------------------
# instancing
# ----------------------------------------------------------------------------
class _Blas(C.Structure):
    _fields_ = [("verts", C.c_void_p), ("n_tris", C.c_uint32), ("nodes", C.c_void_p),
                ("perm", C.c_void_p), ("geom", C.c_void_p), ("texcoords", C.c_void_p)]


class _Inst(C.Structure):
    _fields_ = [("blas", C.c_uint32), ("m", C.c_float * 12)]


def _instance_args(blas_vertices, blas_bvhs, inst_blas, inst_m, geom_ids=None, texcoords=None):
    """geom_ids / texcoords: per-mesh lists (alpha intersector) or None."""
    keep = []
    blas = (_Blas * len(blas_vertices))()
    for i, (v, b) in enumerate(zip(blas_vertices, blas_bvhs)):
        vv = np.ascontiguousarray(v, np.float32).reshape(-1, 9)
        keep += [vv, b.nodes, b.perm]
        blas[i].verts = vv.ctypes.data
        blas[i].n_tris = vv.shape[0]
        blas[i].nodes = b.nodes.ctypes.data
        blas[i].perm = b.perm.ctypes.data
        if geom_ids is not None and geom_ids[i] is not None:
            g = np.ascontiguousarray(geom_ids[i], np.uint32)
            if g.shape[0] < vv.shape[0]:
                raise ValueError("geom_ids must cover every triangle of the mesh")
            keep.append(g)
            blas[i].geom = g.ctypes.data
        if texcoords is not None and texcoords[i] is not None:
            tc = np.ascontiguousarray(texcoords[i], np.float32)
            if tc.shape[0] < vv.shape[0]:
                raise ValueError("texcoords must cover every triangle of the mesh")
            keep.append(tc)
            blas[i].texcoords = tc.ctypes.data
    n = len(inst_blas)
    inst = (_Inst * max(1, n))()
    m = np.ascontiguousarray(inst_m, np.float32).reshape(-1, 12)
    for j in range(n):
        inst[j].blas = int(inst_blas[j])
        inst[j].m[:] = m[j].tolist()
    return blas, inst, keep


def build_tlas(world_lo, world_hi) -> OracleBVH:
    """Top-level BVH over instance world boxes (each as the degenerate
    triangle lo, hi, hi)."""
    lo = np.asarray(world_lo, np.float32)
    hi = np.asarray(world_hi, np.float32)
    return build_bvh(np.stack([lo, hi, hi], axis=1))


def brute_instanced(blas_vertices, inst_blas, inst_m, rays, kind="default", checker_n=8, *,
                    geom_ids=None, texcoords=None, textures=None, alpha_min=128):
    """float64 definition over every instance and triangle.  Alpha: per-mesh
    geom_ids and texcoords lists, one shared texture array.  Returns ``t, u,
    v, prim, inst, flags`` and the float32 error bounds ``bound_uv, bound_t``
    of the nearest hit (the single-scene bound plus the object-ray
    transform's rounding)."""
    lib = _load()
    bvhs = [OracleBVH(np.zeros(1, NODE_DTYPE), np.zeros(1, np.uint32), 0)] * len(blas_vertices)
    blas, inst, keep = _instance_args(blas_vertices, bvhs, inst_blas, inst_m, geom_ids, texcoords)
    r = np.ascontiguousarray(rays, np.float32).reshape(-1, 8)
    m = r.shape[0]
    out = {k: np.empty(m, np.float64) for k in ("t", "u", "v", "bound_uv", "bound_t")}
    out["prim"] = np.empty(m, np.uint32)
    out["inst"] = np.empty(m, np.uint32)
    out["flags"] = np.empty(m, np.uint8)
    if kind == "alpha" and (textures is None or texcoords is None):
        raise ValueError("alpha intersector needs per-mesh texcoords and a texture array")
    is_, k2 = _isect(None, textures, alpha_min, checker_n)
    rc = lib.orc_brute_instanced(blas, len(blas_vertices), inst, len(inst_blas), _ptr(r), m,
                                 KINDS[kind], C.byref(is_), _ptr(out["t"]), _ptr(out["prim"]),
                                 _ptr(out["inst"]), _ptr(out["u"]), _ptr(out["v"]),
                                 _ptr(out["flags"]), _ptr(out["bound_uv"]),
                                 _ptr(out["bound_t"]))
    if rc != 0:
        raise RuntimeError(f"orc_brute_instanced failed ({rc})")
    del keep, k2
    return out


def traverse_instanced(blas_vertices, blas_bvhs, inst_blas, inst_m, tlas: OracleBVH, rays,
                       kind="default", checker_n=8, any_hit=False, count=True, *,
                       geom_ids=None, texcoords=None, textures=None, alpha_min=128):
    """float32 two-level traversal (oracle B).  Alpha: per-mesh geom_ids and
    texcoords lists, one shared texture array."""
    lib = _load()
    blas, inst, keep = _instance_args(blas_vertices, blas_bvhs, inst_blas, inst_m, geom_ids,
                                      texcoords)
    r = np.ascontiguousarray(rays, np.float32).reshape(-1, 8)
    m = r.shape[0]
    out = {k: np.empty(m, np.float32) for k in ("t", "u", "v")}
    out["prim"] = np.empty(m, np.uint32)
    out["inst"] = np.empty(m, np.uint32)
    cnt = np.empty((m, 4), np.uint32) if count else None
    if kind == "alpha" and (textures is None or texcoords is None):
        raise ValueError("alpha intersector needs per-mesh texcoords and a texture array")
    is_, k2 = _isect(None, textures, alpha_min, checker_n)
    rc = lib.orc_traverse_instanced(blas, len(blas_vertices), inst, len(inst_blas),
                                    _ptr(tlas.nodes), _ptr(tlas.perm), _ptr(r), m, KINDS[kind],
                                    C.byref(is_), int(bool(any_hit)), _ptr(out["t"]),
                                    _ptr(out["prim"]), _ptr(out["inst"]), _ptr(out["u"]),
                                    _ptr(out["v"]), _ptr(cnt))
    if rc != 0:
        raise RuntimeError(f"orc_traverse_instanced failed ({rc})")
    if count:
        out["counters"] = cnt
    del keep, k2
    return out
