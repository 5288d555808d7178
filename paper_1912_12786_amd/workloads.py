"""Seeded synthetic scenes, textures and rays.

This module only *draws inputs*: it holds no ray/box/triangle test, no BVH
logic and no intersector.  Both the GPU path and the CPU oracle receive the
arrays it returns, so it is the one module the two sides share.

The paper (Section 4 and the teaser figure) shows alpha-masked billboards,
a procedural alpha mask and a BVH-cost heat map on unnamed 3-d models; those
models are not available, so the scenes below are synthetic stand-ins with the
same structure:

* ``tiny``        -- 1,024 small random triangles in the unit cube, 64x64 rays.
* ``billboards``  -- 100k camera-facing textured quads (200k triangles),
                     16 RGBA8 256x256 alpha textures (about 40 % zero texels),
                     1920x1080 primary rays.
* ``spheres``     -- 2,000 UV-spheres of 500 triangles (1M triangles),
                     1920x1080 primary rays plus incoherent diffuse bounce rays.

All randomness comes from ``numpy.random.Generator(PCG64(seed))`` with
``seed = 191212786 + 1000 * config + stream``; geometry is generated in float64
and rounded once to float32.

Array conventions (shared by every consumer):

* vertices  ``float32 [n_tris, 3, 3]`` (triangle, corner, xyz)
* rays      ``float32 [n_rays, 8]`` = ``(ox, oy, oz, tmin, dx, dy, dz, tmax)``
* texcoords ``float32 [n_tris, 3, 2]`` indexed by the input triangle index
* textures  ``uint32  [n_tex, H, W]`` RGBA8 packed with R in the low byte and
            alpha in the high byte
* geom_ids  ``uint32  [n_tris]``
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 191212786

CFG_TINY = 1
CFG_BILLBOARDS = 2
CFG_SPHERES = 3
CFG_BATCHED = 4
CFG_DIFF = 5

STREAM_GEOMETRY = 0
STREAM_TEXTURES = 1
STREAM_RAYS = 2
STREAM_WEIGHTS = 3


def seed_for(config: int, stream: int) -> int:
    return SEED_BASE + 1000 * config + stream


def rng_for(config: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed_for(config, stream)))


# --------------------------------------------------------------------------
# small vector helpers (input synthesis only)
# --------------------------------------------------------------------------
def _normalize(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _random_unit(rng: np.random.Generator, n: int) -> np.ndarray:
    return _normalize(rng.standard_normal((n, 3)))


def _onb_from_normal(n: np.ndarray):
    """Branchless orthonormal basis around unit vectors n (Duff et al. 2017)."""
    sign = np.where(n[:, 2] >= 0.0, 1.0, -1.0)
    a = -1.0 / (sign + n[:, 2])
    b = n[:, 0] * n[:, 1] * a
    t = np.stack([1.0 + sign * n[:, 0] ** 2 * a, sign * b, -sign * n[:, 0]], axis=1)
    bt = np.stack([b, sign + n[:, 1] ** 2 * a, -n[:, 1]], axis=1)
    return t, bt


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------
def pinhole_rays(width: int, height: int, eye, center, fov_deg: float,
                 tmin: float = 0.0, tmax: float = math.inf) -> np.ndarray:
    """Primary rays of a pinhole camera, scanline order, row 0 at the top.

    ``fov_deg`` is the vertical field of view.  Returns ``float32 [W*H, 8]``.
    """
    eye = np.asarray(eye, np.float64)
    center = np.asarray(center, np.float64)
    fwd = _normalize(center - eye)
    right = _normalize(np.cross(fwd, np.array([0.0, 1.0, 0.0])))
    up = np.cross(right, fwd)
    th = math.tan(math.radians(fov_deg) / 2.0)
    xs = (2.0 * (np.arange(width) + 0.5) / width - 1.0) * th * width / height
    ys = (1.0 - 2.0 * (np.arange(height) + 0.5) / height) * th
    d = (fwd[None, None, :] + xs[None, :, None] * right[None, None, :]
         + ys[:, None, None] * up[None, None, :])
    d = _normalize(d.reshape(-1, 3))
    rays = np.empty((width * height, 8), np.float32)
    rays[:, 0:3] = eye.astype(np.float32)
    rays[:, 3] = np.float32(tmin)
    rays[:, 4:7] = d.astype(np.float32)
    rays[:, 7] = np.float32(tmax)
    return rays


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------
def random_triangles(n: int, seed: int, side: float = 0.05,
                     box=(0.0, 1.0)) -> np.ndarray:
    """Equilateral triangles with side ``side``, centres uniform in ``box``^3,
    random plane and spin."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.uniform(box[0], box[1], size=(n, 3))
    a = _random_unit(rng, n)
    g = _random_unit(rng, n)
    b = np.cross(a, g)
    bn = np.linalg.norm(b, axis=1, keepdims=True)
    # a degenerate draw (g parallel to a) is replaced deterministically
    bad = (bn[:, 0] < 1e-6)
    if bad.any():
        alt = np.cross(a[bad], np.array([0.0, 0.0, 1.0]))
        b[bad] = alt
        bn[bad] = np.linalg.norm(alt, axis=1, keepdims=True)
    b = b / bn
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n)
    r = side / math.sqrt(3.0)
    v = np.empty((n, 3, 3), np.float64)
    for k in range(3):
        th = phi + 2.0 * math.pi * k / 3.0
        v[:, k, :] = c + r * (np.cos(th)[:, None] * a + np.sin(th)[:, None] * b)
    return v.astype(np.float32)


def billboard_quads(n_quads: int, seed: int, eye, n_tex: int = 16,
                    box=(0.0, 100.0), side=(0.5, 2.0)):
    """Camera-facing textured quads, two triangles each.

    Quad ``q`` becomes triangles ``2q = (c00, c10, c11)`` and
    ``2q+1 = (c00, c11, c01)`` with texture coordinates
    ``(0,0),(1,0),(1,1)`` and ``(0,0),(1,1),(0,1)``.
    Returns ``(vertices, texcoords, geom_ids)``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    eye = np.asarray(eye, np.float64)
    c = rng.uniform(box[0], box[1], size=(n_quads, 3))
    s = rng.uniform(side[0], side[1], size=n_quads)
    tex_of_quad = rng.integers(0, n_tex, size=n_quads, dtype=np.int64)
    n = _normalize(eye[None, :] - c)
    right = _normalize(np.cross(np.array([0.0, 1.0, 0.0])[None, :], n))
    up = np.cross(n, right)
    h = (s / 2.0)[:, None]
    c00 = c - h * right - h * up
    c10 = c + h * right - h * up
    c11 = c + h * right + h * up
    c01 = c - h * right + h * up
    v = np.empty((2 * n_quads, 3, 3), np.float64)
    v[0::2, 0], v[0::2, 1], v[0::2, 2] = c00, c10, c11
    v[1::2, 0], v[1::2, 1], v[1::2, 2] = c00, c11, c01
    tc = np.empty((2 * n_quads, 3, 2), np.float32)
    tc[0::2] = np.array([[0, 0], [1, 0], [1, 1]], np.float32)
    tc[1::2] = np.array([[0, 0], [1, 1], [0, 1]], np.float32)
    geom = np.repeat(tex_of_quad, 2).astype(np.uint32)
    return v.astype(np.float32), tc, geom


def uv_sphere(center, radius: float, slices: int = 25, stacks: int = 11) -> np.ndarray:
    """Triangles of a UV-sphere: two polar fans plus quad bands.

    ``2*slices*(stacks-1)`` triangles (500 for the defaults)."""
    center = np.asarray(center, np.float64)
    th = math.pi * np.arange(1, stacks) / stacks          # ring polar angles
    ph = 2.0 * math.pi * np.arange(slices) / slices
    ring = np.stack([np.sin(th)[:, None] * np.cos(ph)[None, :],
                     np.cos(th)[:, None] * np.ones_like(ph)[None, :],
                     np.sin(th)[:, None] * np.sin(ph)[None, :]], axis=-1)
    ring = center + radius * ring                          # [stacks-1, slices, 3]
    north = center + radius * np.array([0.0, 1.0, 0.0])
    south = center - radius * np.array([0.0, 1.0, 0.0])
    tris = []
    j = np.arange(slices)
    jn = (j + 1) % slices
    tris.append(np.stack([np.broadcast_to(north, (slices, 3)), ring[0, j], ring[0, jn]], 1))
    for i in range(stacks - 2):
        a, b = ring[i], ring[i + 1]
        tris.append(np.stack([a[j], b[j], b[jn]], 1))
        tris.append(np.stack([a[j], b[jn], a[jn]], 1))
    tris.append(np.stack([ring[-1, j], np.broadcast_to(south, (slices, 3)), ring[-1, jn]], 1))
    return np.concatenate(tris, 0)


def sphere_scene(n_spheres: int, seed: int, box=(0.0, 100.0),
                 radius=(0.1, 5.0), slices: int = 25, stacks: int = 11):
    """Random UV-spheres; radii log-uniform.  Returns (vertices, centres, radii)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.uniform(box[0], box[1], size=(n_spheres, 3))
    r = np.exp(rng.uniform(math.log(radius[0]), math.log(radius[1]), size=n_spheres))
    unit = uv_sphere(np.zeros(3), 1.0, slices, stacks)     # [T, 3, 3]
    v = c[:, None, None, :] + r[:, None, None, None] * unit[None]
    return v.reshape(-1, 3, 3).astype(np.float32), c, r


def sphere_bounce_rays(n: int, centres: np.ndarray, radii: np.ndarray,
                       eye, seed: int) -> np.ndarray:
    """Incoherent secondary rays leaving sphere surfaces.

    A sphere is drawn with probability proportional to its cross-section
    (radius squared), a point on its camera-facing hemisphere is drawn
    uniformly, the origin is placed 1e-4 radii outside the analytic sphere
    (the tessellation is inscribed, so the origin is outside the mesh), and
    the direction is cosine-weighted about the outward normal (Malley's
    method).  A ray leaving a convex body through its outward hemisphere never
    re-enters it, so no self-intersection is possible.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    eye = np.asarray(eye, np.float64)
    p = radii ** 2
    p = p / p.sum()
    k = rng.choice(len(radii), size=n, p=p)
    w = _random_unit(rng, n)
    view = eye[None, :] - centres[k]
    flip = np.sum(w * view, axis=1) < 0.0
    w[flip] = -w[flip]
    org = centres[k] + (radii[k] * (1.0 + 1e-4))[:, None] * w
    xi1 = rng.uniform(0.0, 1.0, size=n)
    xi2 = rng.uniform(0.0, 1.0, size=n)
    rr = np.sqrt(xi1)
    ph = 2.0 * math.pi * xi2
    lx, ly = rr * np.cos(ph), rr * np.sin(ph)
    lz = np.sqrt(np.maximum(0.0, 1.0 - xi1))
    t, bt = _onb_from_normal(w)
    d = _normalize(lx[:, None] * t + ly[:, None] * bt + lz[:, None] * w)
    rays = np.empty((n, 8), np.float32)
    rays[:, 0:3] = org.astype(np.float32)
    rays[:, 3] = 0.0
    rays[:, 4:7] = d.astype(np.float32)
    rays[:, 7] = np.inf
    return rays


# --------------------------------------------------------------------------
# alpha textures
# --------------------------------------------------------------------------
def alpha_textures(n_tex: int, size: int, seed: int, target_nonzero: float = 0.60,
                   tol: float = 0.02) -> np.ndarray:
    """RGBA8 textures whose alpha holds seeded disks and soft Gaussian blobs.

    Alpha starts at zero; opaque disks (radius U[6,40] px) and blobs (sums of
    3-6 Gaussians, alpha = round(255*min(1, g))) are added one at a time until
    the fraction of non-zero alpha texels reaches ``target_nonzero - tol``; a
    shape that would push it above ``target_nonzero + tol`` is redrawn.
    RGB is uniform random.  Returns ``uint32 [n_tex, size, size]``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    yy, xx = np.mgrid[0:size, 0:size].astype(np.float64)
    out = np.empty((n_tex, size, size), np.uint32)
    for ti in range(n_tex):
        alpha = np.zeros((size, size), np.float64)
        frac = 0.0
        attempts = 0
        while frac < target_nonzero - tol and attempts < 10000:
            attempts += 1
            cand = alpha.copy()
            if rng.uniform() < 0.5:
                cx, cy = rng.uniform(0, size, size=2)
                rad = rng.uniform(6.0, 40.0)
                cand[(xx - cx) ** 2 + (yy - cy) ** 2 <= rad * rad] = 1.0
            else:
                bx, by = rng.uniform(0, size, size=2)
                g = np.zeros_like(alpha)
                for _ in range(int(rng.integers(3, 7))):
                    gx, gy = bx + rng.uniform(-20, 20), by + rng.uniform(-20, 20)
                    sg = rng.uniform(4.0, 16.0)
                    amp = rng.uniform(0.5, 1.5)
                    g += amp * np.exp(-((xx - gx) ** 2 + (yy - gy) ** 2) / (2.0 * sg * sg))
                cand = np.maximum(cand, np.minimum(1.0, g))
            cfrac = float(np.mean(np.round(255.0 * cand) > 0))
            if cfrac > target_nonzero + tol:
                continue
            alpha, frac = cand, cfrac
        a8 = np.round(255.0 * np.minimum(1.0, alpha)).astype(np.uint32)
        rgb = rng.integers(0, 256, size=(size, size, 3), dtype=np.uint32)
        out[ti] = rgb[..., 0] | (rgb[..., 1] << 8) | (rgb[..., 2] << 16) | (a8 << 24)
    return out


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    vertices: np.ndarray                 # float32 [n, 3, 3]
    rays: np.ndarray                     # float32 [N, 8]
    geom_ids: np.ndarray | None = None   # uint32 [n]
    texcoords: np.ndarray | None = None  # float32 [n, 3, 2]
    textures: np.ndarray | None = None   # uint32 [n_tex, H, W]
    extra: dict = field(default_factory=dict)

    @property
    def n_tris(self) -> int:
        return int(self.vertices.shape[0])

    @property
    def n_rays(self) -> int:
        return int(self.rays.shape[0])


BILLBOARD_EYE = (50.0, 50.0, -60.0)
BILLBOARD_CENTER = (50.0, 50.0, 50.0)


def tiny(width: int = 64, height: int = 64) -> Workload:
    """1,024 random triangles (side 0.05) in the unit cube; 64x64 primary rays
    from distance 2, vertical fov 40 degrees."""
    v = random_triangles(1024, seed_for(CFG_TINY, STREAM_GEOMETRY))
    rays = pinhole_rays(width, height, (0.5, 0.5, 2.5), (0.5, 0.5, 0.5), 40.0)
    return Workload(f"tiny_1k_tris_{width}x{height}", v, rays,
                    geom_ids=np.zeros(v.shape[0], np.uint32),
                    extra={"width": width, "height": height})


def billboards(n_quads: int = 100_000, width: int = 1920, height: int = 1080,
               n_tex: int = 16, tex_size: int = 256) -> Workload:
    """Alpha-masked billboards: camera-facing quads with RGBA8 alpha masks."""
    v, tc, geom = billboard_quads(n_quads, seed_for(CFG_BILLBOARDS, STREAM_GEOMETRY),
                                  BILLBOARD_EYE, n_tex=n_tex)
    tex = alpha_textures(n_tex, tex_size, seed_for(CFG_BILLBOARDS, STREAM_TEXTURES))
    rays = pinhole_rays(width, height, BILLBOARD_EYE, BILLBOARD_CENTER, 60.0)
    return Workload(f"billboards_{2 * n_quads}_tris_{width}x{height}", v, rays,
                    geom_ids=geom, texcoords=tc, textures=tex,
                    extra={"width": width, "height": height})


def spheres(n_spheres: int = 2000, width: int = 1920, height: int = 1080,
            bounce_fraction: float = 0.8) -> Workload:
    """Tessellated random spheres; primary rays plus diffuse bounce rays.

    ``extra['n_primary']`` rays come first, then the bounce rays.  The bounce
    count is ``bounce_fraction`` of the primary count (about the fraction of
    primary rays that hit a sphere in this scene)."""
    v, c, r = sphere_scene(n_spheres, seed_for(CFG_SPHERES, STREAM_GEOMETRY))
    prim = pinhole_rays(width, height, BILLBOARD_EYE, BILLBOARD_CENTER, 60.0)
    nb = int(round(bounce_fraction * prim.shape[0]))
    bounce = sphere_bounce_rays(nb, c, r, BILLBOARD_EYE, seed_for(CFG_SPHERES, STREAM_RAYS))
    rays = np.concatenate([prim, bounce], 0)
    return Workload(f"spheres_{v.shape[0]}_tris_{width}x{height}_plus_bounce", v, rays,
                    geom_ids=np.zeros(v.shape[0], np.uint32),
                    extra={"n_primary": prim.shape[0], "centres": c, "radii": r,
                           "width": width, "height": height})


def subsample_indices(n_rays: int, width: int | None, height: int | None,
                      seed: int, stride: int = 8, n_random: int = 8192) -> np.ndarray:
    """Stratified ray subsample: every ``stride``-th pixel in x and y at a
    seeded offset, plus ``n_random`` uniformly drawn rays (sorted, unique)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = []
    if width is not None and height is not None:
        ox, oy = rng.integers(0, stride, size=2)
        ys = np.arange(oy, height, stride)
        xs = np.arange(ox, width, stride)
        idx.append((ys[:, None] * width + xs[None, :]).ravel())
    idx.append(rng.integers(0, n_rays, size=min(n_random, n_rays)))
    return np.unique(np.concatenate(idx)).astype(np.int64)


# --------------------------------------------------------------------------
# indexed meshes (for the differentiable hit)
# --------------------------------------------------------------------------
def geodesic_sphere(freq: int):
    """Class-I geodesic sphere: each of the icosahedron's 20 faces is cut into
    freq^2 triangles and every vertex is projected to the unit sphere.
    Returns (vertices float64 [10 freq^2 + 2, 3], faces int64 [20 freq^2, 3])."""
    p = (1.0 + math.sqrt(5.0)) / 2.0
    ico_v = np.array([[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
                      [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
                      [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], np.float64)
    ico_f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                      [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                      [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                      [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], np.int64)
    key_to_id: dict = {}
    verts = []

    def vid(a, b, c, i, j):
        # point i/freq along (a->b), j/freq along (a->c); keyed by its exact
        # integer barycentric coordinates on the icosahedron's vertex set
        k = freq - i - j
        coords = {a: k, b: i, c: j}
        key = tuple(sorted((v, w) for v, w in coords.items() if w))
        if key not in key_to_id:
            pt = (k * ico_v[a] + i * ico_v[b] + j * ico_v[c]) / freq
            key_to_id[key] = len(verts)
            verts.append(pt / np.linalg.norm(pt))
        return key_to_id[key]

    faces = []
    for a, b, c in ico_f:
        for i in range(freq):
            for j in range(freq - i):
                faces.append((vid(a, b, c, i, j), vid(a, b, c, i + 1, j), vid(a, b, c, i, j + 1)))
                if i + j < freq - 1:
                    faces.append((vid(a, b, c, i + 1, j), vid(a, b, c, i + 1, j + 1),
                                  vid(a, b, c, i, j + 1)))
    return np.asarray(verts, np.float64), np.asarray(faces, np.int64)


DIFF_EYE = (0.0, 0.0, 4.0)


@dataclass
class MeshWorkload:
    name: str
    vertices: np.ndarray    # float32 [nv, 3]
    faces: np.ndarray       # uint32 [n, 3]
    rays: np.ndarray        # float32 [N, 8]
    geom_ids: np.ndarray    # uint32 [n]
    texcoords: np.ndarray   # float32 [n, 3, 2]
    textures: np.ndarray    # uint32 [n_tex, H, W]
    weights: np.ndarray     # float32 [N, 3] loss weights on (t, u, v)
    opaque_tex: int         # texture id of the sphere (alpha 255 everywhere)

    @property
    def triangles(self) -> np.ndarray:
        return self.vertices[self.faces]


def diff_scene(freq: int = 50, n_billboards: int = 5000, width: int = 512, height: int = 512,
               noise: float = 0.01, n_tex: int = 16, tex_size: int = 256) -> MeshWorkload:
    """Perturbed geodesic sphere (20 freq^2 triangles, radius 1, vertex noise
    N(0, noise^2) per coordinate) plus camera-facing alpha billboards (centres
    in the shell 1.2 <= r <= 2, side U[0.05, 0.2], the billboard textures)
    seen by a width x height pinhole camera at (0, 0, 4) with fov 40 degrees.
    Loss weights on (t, u, v) are uniform in [-1, 1] per ray.  The sphere uses
    an extra fully opaque texture so that one alpha-mask launch covers both."""
    g = rng_for(CFG_DIFF, STREAM_GEOMETRY)
    sv, sf = geodesic_sphere(freq)
    sv = sv + g.normal(0.0, noise, size=sv.shape)
    eye = np.asarray(DIFF_EYE, np.float64)
    dirs = _random_unit(g, n_billboards)
    rad = g.uniform(1.2, 2.0, size=n_billboards)
    c = dirs * rad[:, None]
    s = g.uniform(0.05, 0.2, size=n_billboards)
    n = _normalize(eye[None, :] - c)
    right = _normalize(np.cross(np.array([0.0, 1.0, 0.0])[None, :], n))
    up = np.cross(n, right)
    h = (s / 2.0)[:, None]
    quad = np.stack([c - h * right - h * up, c + h * right - h * up,
                     c + h * right + h * up, c - h * right + h * up], axis=1)   # [q, 4, 3]
    bv = quad.reshape(-1, 3)
    base = sv.shape[0] + 4 * np.arange(n_billboards)
    bf = np.concatenate([np.stack([base, base + 1, base + 2], 1),
                         np.stack([base, base + 2, base + 3], 1)], 0)
    order = np.argsort(np.concatenate([2 * np.arange(n_billboards), 2 * np.arange(n_billboards) + 1]),
                       kind="stable")
    bf = bf[order]                                  # quad q -> faces 2q, 2q+1
    verts = np.concatenate([sv, bv], 0).astype(np.float32)
    faces = np.concatenate([sf, bf], 0).astype(np.uint32)
    tex = alpha_textures(n_tex, tex_size, seed_for(CFG_BILLBOARDS, STREAM_TEXTURES))
    opaque = np.full((1, tex_size, tex_size), np.uint32(0xFF808080), np.uint32)
    textures = np.concatenate([tex, opaque], 0)
    n_sphere = sf.shape[0]
    tc = np.zeros((faces.shape[0], 3, 2), np.float32)
    tc[n_sphere + 0::2] = np.array([[0, 0], [1, 0], [1, 1]], np.float32)
    tc[n_sphere + 1::2] = np.array([[0, 0], [1, 1], [0, 1]], np.float32)
    geom = np.full(faces.shape[0], n_tex, np.uint32)
    geom[n_sphere:] = np.repeat(g.integers(0, n_tex, size=n_billboards), 2).astype(np.uint32)
    rays = pinhole_rays(width, height, DIFF_EYE, (0.0, 0.0, 0.0), 40.0)
    w = rng_for(CFG_DIFF, STREAM_WEIGHTS).uniform(-1.0, 1.0, size=(rays.shape[0], 3)).astype(np.float32)
    return MeshWorkload(f"diff_icosphere_{n_sphere}_plus_{2 * n_billboards}_billboard_tris_{width}x{height}",
                        verts, faces, rays, geom, tc, textures, w, n_tex)


# --------------------------------------------------------------------------
# batched multi-scene workload
# --------------------------------------------------------------------------
def incoherent_rays(n: int, seed: int, box=(0.0, 100.0)) -> np.ndarray:
    """Bounce-like rays: origins uniform in the box, directions uniform on the
    sphere (a stand-in for diffuse secondary rays of any scene type)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    o = rng.uniform(box[0], box[1], size=(n, 3))
    d = _random_unit(rng, n)
    rays = np.empty((n, 8), np.float32)
    rays[:, 0:3] = o.astype(np.float32)
    rays[:, 3] = 0.0
    rays[:, 4:7] = d.astype(np.float32)
    rays[:, 7] = np.inf
    return rays


def batched(n_scenes: int = 64, tri_range=(1_000, 500_000), ray_range=(4_000, 2_000_000),
            width: int = 1920):
    """Scenes of uneven size, each with its own ray batch.

    Triangle and ray counts are log-uniform in the given ranges; the scene
    type cycles through random triangles (rescaled to [0, 100]^3), camera
    facing billboards and tessellated spheres.  Half of each ray batch is
    primary rays of a 1920-wide camera (rows truncated to the count), half
    incoherent rays.  Returns a list of dicts with ``vertices`` and ``rays``."""
    g = rng_for(CFG_BATCHED, STREAM_GEOMETRY)
    n_t = np.exp(g.uniform(math.log(tri_range[0]), math.log(tri_range[1]), size=n_scenes))
    n_r = np.exp(g.uniform(math.log(ray_range[0]), math.log(ray_range[1]), size=n_scenes))
    out = []
    for s in range(n_scenes):
        seed = seed_for(CFG_BATCHED, 100 + s)
        kind = s % 3
        nt = int(n_t[s])
        if kind == 0:
            v = random_triangles(nt, seed, side=5.0, box=(0.0, 100.0))
        elif kind == 1:
            v, _, _ = billboard_quads(max(1, nt // 2), seed, BILLBOARD_EYE)
        else:
            v, _, _ = sphere_scene(max(1, nt // 500), seed)
        nr = int(n_r[s])
        n_prim = nr // 2
        height = max(1, -(-n_prim // width))
        prim = pinhole_rays(width, height, BILLBOARD_EYE, BILLBOARD_CENTER, 60.0)[:n_prim]
        rays = np.concatenate([prim, incoherent_rays(nr - n_prim, seed + 1)], 0)
        out.append({"vertices": v, "rays": rays, "type": ("triangles", "billboards", "spheres")[kind]})
    return out


# --------------------------------------------------------------------------
# instanced scenes
# --------------------------------------------------------------------------
def _rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def instance_transforms(world_from_object: np.ndarray, blas_lo: np.ndarray, blas_hi: np.ndarray):
    """For row-major 3x4 world-from-object maps (float64 [n, 3, 4]) and each
    instance's object-space box: the object-from-world maps rounded to float32
    ([n, 12]) and world boxes (float32) that contain the instance under that
    rounded map -- the 8 transformed corners, padded outward by 1e-5 of the
    extent."""
    n = world_from_object.shape[0]
    L = world_from_object[:, :, :3]
    T = world_from_object[:, :, 3]
    Linv = np.linalg.inv(L)
    ofw = np.concatenate([Linv, -np.einsum("nij,nj->ni", Linv, T)[..., None]], axis=2)
    corners = np.stack(np.meshgrid([0, 1], [0, 1], [0, 1], indexing="ij"), -1).reshape(8, 3)
    c = blas_lo[:, None, :] + corners[None] * (blas_hi - blas_lo)[:, None, :]      # [n, 8, 3]
    w = np.einsum("nij,nkj->nki", L, c) + T[:, None, :]
    lo, hi = w.min(1), w.max(1)
    pad = 1e-5 * (hi - lo).max(1, keepdims=True) + 1e-6
    lo32 = np.nextafter((lo - pad).astype(np.float32), np.float32(-np.inf))
    hi32 = np.nextafter((hi + pad).astype(np.float32), np.float32(np.inf))
    return ofw.reshape(n, 12).astype(np.float32), lo32, hi32


def tight_world_boxes(world_from_object: np.ndarray, meshes, ids: np.ndarray):
    """World boxes of instances from their transformed vertices (tighter than
    the transformed object box of a rotated instance), padded outward by
    1e-5 of the extent and rounded outward to float32, like
    instance_transforms()."""
    n = world_from_object.shape[0]
    lo = np.zeros((n, 3))
    hi = np.zeros((n, 3))
    for q in range(n):
        v = np.asarray(meshes[ids[q]], np.float64).reshape(-1, 3)
        if v.size == 0:
            lo[q] = hi[q] = world_from_object[q, :, 3]
            continue
        w = v @ world_from_object[q, :, :3].T + world_from_object[q, :, 3]
        lo[q], hi[q] = w.min(0), w.max(0)
    pad = 1e-5 * (hi - lo).max(1, keepdims=True) + 1e-6
    lo32 = np.nextafter((lo - pad).astype(np.float32), np.float32(-np.inf))
    hi32 = np.nextafter((hi + pad).astype(np.float32), np.float32(np.inf))
    return lo32, hi32


def instanced(n_instances: int = 2000, width: int = 1920, height: int = 1080):
    """Object instancing: three meshes (a 500-triangle sphere, 500 random
    triangles, 50 billboard quads) instanced n_instances times with random
    rotations, scales in [0.5, 3] and positions uniform in [0, 100]^3, seen by
    the billboard camera.  Returns dict with blas vertex lists, per-instance
    blas ids, object-from-world maps, world boxes (from the transformed
    vertices) and rays."""
    g = rng_for(CFG_BATCHED, 900)
    blas = [uv_sphere(np.zeros(3), 1.0).astype(np.float32),
            random_triangles(500, seed_for(CFG_BATCHED, 901), side=0.3, box=(-1.0, 1.0)),
            billboard_quads(50, seed_for(CFG_BATCHED, 902), (0.0, 0.0, -10.0),
                            box=(-1.0, 1.0), side=(0.2, 0.6))[0]]
    ids = g.integers(0, len(blas), size=n_instances).astype(np.uint32)
    wfo = np.empty((n_instances, 3, 4))
    for i in range(n_instances):
        wfo[i, :, :3] = _rotation(g) * g.uniform(0.5, 3.0)
        wfo[i, :, 3] = g.uniform(0.0, 100.0, size=3)
    blo = np.stack([b.reshape(-1, 3).min(0) for b in blas]).astype(np.float64)[ids]
    bhi = np.stack([b.reshape(-1, 3).max(0) for b in blas]).astype(np.float64)[ids]
    m, _, _ = instance_transforms(wfo, blo, bhi)
    lo, hi = tight_world_boxes(wfo, blas, ids)
    rays = pinhole_rays(width, height, BILLBOARD_EYE, BILLBOARD_CENTER, 60.0)
    return {"blas": blas, "inst_blas": ids, "inst_m": m, "world_lo": lo, "world_hi": hi,
            "rays": rays, "world_from_object": wfo, "width": width, "height": height,
            "name": f"instanced_{n_instances}_x3_meshes_{width}x{height}"}


def instanced_alpha(wl, n_tex: int = 16, tex_size: int = 256) -> dict:
    """Alpha-mask inputs for an ``instanced`` workload: in every mesh each pair
    of consecutive triangles gets one texture id in U{0..n_tex-1} and the
    billboard texture coordinates ``(0,0),(1,0),(1,1)`` / ``(0,0),(1,1),(0,1)``;
    the textures are the billboard workload's.  Returns the keyword arguments
    of ``InstancedScene`` (``geom_ids``, ``texcoords``, ``textures``)."""
    g = rng_for(CFG_BATCHED, 903)
    geoms, tcs = [], []
    for mesh in wl["blas"]:
        n = int(mesh.shape[0])
        geoms.append(np.repeat(g.integers(0, n_tex, size=(n + 1) // 2), 2)[:n].astype(np.uint32))
        tc = np.empty((n, 3, 2), np.float32)
        tc[0::2] = np.array([[0, 0], [1, 0], [1, 1]], np.float32)
        tc[1::2] = np.array([[0, 0], [1, 1], [0, 1]], np.float32)
        tcs.append(tc)
    tex = alpha_textures(n_tex, tex_size, seed_for(CFG_BILLBOARDS, STREAM_TEXTURES))
    return {"geom_ids": geoms, "texcoords": tcs, "textures": tex}
