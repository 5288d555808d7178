// rt_traverse.hpp -- device-side BVH traversal with compile-time intersectors
// for gfx950 (HIP, wave64).
//
// The custom-intersector method (Sections 3.1-3.2): the two intersect calls
// of the while-while BVH traversal (Algorithm 1) -- ray vs. node bounds and
// ray vs. primitive -- are statically replaced by the intersector's member
// functions.  Here an intersector is any type with these members (each has a
// default in intersector_base, so a user type only writes what it changes):
//
//   void on_box_test()                 every ray/box test (Listing 6, aabb overload)
//   void on_tri_test()                 every ray/triangle test (Listing 6)
//   bool accept(const hit_candidate&)  decides a geometric hit inside the
//                                      current interval; the result is AND-ed
//                                      into the hit (Listing 3: hr.hit &= ...)
//   static constexpr bool kFilters     false lets the traversal skip the
//                                      accept call entirely (zero cost when no
//                                      custom code is supplied, Section 1)
//
// The intersector object lives in registers for one ray, so per-ray state such
// as the heat-map counters of Listing 6 is plain member data.
//
// All floating-point work is float32 and bit-reproducible: fused
// multiply-adds are explicit fmaf() calls (the library is compiled with
// -ffp-contract=off), divisions are IEEE divisions, and min/max are exact.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtx {

// -------------------------------------------------------------------------
// records in device memory (layouts documented with the builder)
// -------------------------------------------------------------------------
constexpr uint32_t kRefIndexMask = 0x1FFFFFFFu;
constexpr uint32_t kMissPrim = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t ref_count(uint32_t ref) { return ref >> 29; }
__device__ __forceinline__ uint32_t ref_index(uint32_t ref) { return ref & kRefIndexMask; }

struct hit_candidate {
    uint32_t prim_id;  // input index of the triangle
    uint32_t geom_id;
    float t, u, v;
};

// -------------------------------------------------------------------------
// intersectors
// -------------------------------------------------------------------------
struct intersector_base {
    static constexpr bool kFilters = false;
    static constexpr bool kCounts = false;
    __device__ __forceinline__ void on_box_test() {}
    __device__ __forceinline__ void on_tri_test() {}
    __device__ __forceinline__ bool accept(const hit_candidate &) { return true; }
};

// Default: every geometric hit is a hit.
struct default_intersector : intersector_base {
    struct params {};
    __device__ explicit default_intersector(const params &) {}
};

// Alpha mask (Section 4, Listing 5): interpolate the triangle's texture
// coordinates with weights (1-u-v, u, v), fetch the nearest texel of texture
// geom_id (clamp to edge) and keep the hit iff its alpha byte reaches
// alpha_min.
struct alpha_intersector : intersector_base {
    static constexpr bool kFilters = true;
    struct params {
        const float2 *texcoords;   // [n_prims][3]
        const uint32_t *textures;  // [n_tex][height][width] RGBA8
        uint32_t width, height, alpha_min;
    };
    params p;
    __device__ explicit alpha_intersector(const params &pp) : p(pp) {}

    __device__ __forceinline__ bool accept(const hit_candidate &c)
    {
        const float2 *tc = p.texcoords + 3 * size_t(c.prim_id);
        const float2 tc0 = tc[0], tc1 = tc[1], tc2 = tc[2];
        const float w0 = (1.0f - c.u) - c.v;
        const float s = fmaf(c.v, tc2.x, fmaf(c.u, tc1.x, w0 * tc0.x));
        const float t = fmaf(c.v, tc2.y, fmaf(c.u, tc1.y, w0 * tc0.y));
        const float xf = fminf(fmaxf(floorf(s * float(p.width)), 0.0f), float(p.width - 1));
        const float yf = fminf(fmaxf(floorf(t * float(p.height)), 0.0f), float(p.height - 1));
        const size_t idx = (size_t(c.geom_id) * p.height + uint32_t(yf)) * p.width + uint32_t(xf);
        return (p.textures[idx] >> 24) >= p.alpha_min;
    }
};

// Procedural alpha mask (Section 4): a checker over the barycentrics,
// visible iff floor(n u) + floor(n v) is even.
struct checker_intersector : intersector_base {
    static constexpr bool kFilters = true;
    struct params {
        uint32_t n;
    };
    float n;
    __device__ explicit checker_intersector(const params &pp) : n(float(pp.n)) {}

    __device__ __forceinline__ bool accept(const hit_candidate &c)
    {
        const int a = int(floorf(n * c.u));
        const int b = int(floorf(n * c.v));
        return ((a + b) & 1) == 0;
    }
};

// Heat-map intersector (Section 4, Listing 6) composed with another one:
// counts the box and triangle tests and the accept decisions, and forwards
// the decision itself to Inner.
template <class Inner>
struct counting_intersector : Inner {
    static constexpr bool kFilters = true;
    static constexpr bool kCounts = true;
    uint32_t num_boxes = 0, num_tris = 0, num_candidates = 0, num_accepted = 0;
    __device__ explicit counting_intersector(const typename Inner::params &pp) : Inner(pp) {}
    __device__ __forceinline__ void on_box_test() { ++num_boxes; }
    __device__ __forceinline__ void on_tri_test() { ++num_tris; }
    __device__ __forceinline__ bool accept(const hit_candidate &c)
    {
        ++num_candidates;
        bool ok = true;
        if constexpr (Inner::kFilters) ok = Inner::accept(c);
        num_accepted += ok ? 1u : 0u;
        return ok;
    }
};

// -------------------------------------------------------------------------
// float32 ray, box and triangle tests
// -------------------------------------------------------------------------
struct ray_state {
    float ox, oy, oz, tmin;
    float dx, dy, dz, tmax;  // tmax shrinks to the nearest accepted hit
    float ix, iy, iz;        // 1/d (with tiny components replaced by +-2^-80)
    float bx, by, bz;        // o * (1/d)
};

__device__ __forceinline__ float safe_inverse(float d)
{
    const float tiny = 0x1p-80f;
    const float dd = fabsf(d) < tiny ? copysignf(tiny, d) : d;
    return 1.0f / dd;
}

__device__ __forceinline__ ray_state make_ray(float4 a, float4 b)
{
    ray_state r;
    r.ox = a.x; r.oy = a.y; r.oz = a.z; r.tmin = a.w;
    r.dx = b.x; r.dy = b.y; r.dz = b.z; r.tmax = b.w;
    r.ix = safe_inverse(b.x);
    r.iy = safe_inverse(b.y);
    r.iz = safe_inverse(b.z);
    r.bx = a.x * r.ix;
    r.by = a.y * r.iy;
    r.bz = a.z * r.iz;
    return r;
}

// Slab test of [lo, hi] over [tmin, tmax]: hit iff tn <= tf (closed, so that
// flat boxes of axis-aligned geometry are hit).
__device__ __forceinline__ bool slab(const ray_state &r, float lx, float ly, float lz,
                                     float hx, float hy, float hz, float &tn)
{
    const float t0x = fmaf(lx, r.ix, -r.bx), t1x = fmaf(hx, r.ix, -r.bx);
    const float t0y = fmaf(ly, r.iy, -r.by), t1y = fmaf(hy, r.iy, -r.by);
    const float t0z = fmaf(lz, r.iz, -r.bz), t1z = fmaf(hz, r.iz, -r.bz);
    tn = fmaxf(fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fminf(t0z, t1z)), r.tmin);
    const float tf = fminf(fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fmaxf(t0z, t1z)), r.tmax);
    return tn <= tf;
}

__device__ __forceinline__ float dot3(float ax, float ay, float az, float bx, float by, float bz)
{
    return fmaf(az, bz, fmaf(ay, by, ax * bx));
}

// Moller-Trumbore, two-sided, closed triangle; returns true iff the hit lies
// strictly inside (tmin, tmax).
__device__ __forceinline__ bool triangle(const ray_state &r, float4 a, float4 b, float4 c,
                                         float &t, float &u, float &v)
{
    // a = {v0, prim}, b = {e1, geom}, c = {e2, 0}
    const float px = fmaf(r.dy, c.z, -(r.dz * c.y));
    const float py = fmaf(r.dz, c.x, -(r.dx * c.z));
    const float pz = fmaf(r.dx, c.y, -(r.dy * c.x));
    const float det = dot3(b.x, b.y, b.z, px, py, pz);
    const float inv = 1.0f / det;
    const float sx = r.ox - a.x, sy = r.oy - a.y, sz = r.oz - a.z;
    u = dot3(sx, sy, sz, px, py, pz) * inv;
    const float qx = fmaf(sy, b.z, -(sz * b.y));
    const float qy = fmaf(sz, b.x, -(sx * b.z));
    const float qz = fmaf(sx, b.y, -(sy * b.x));
    v = dot3(r.dx, r.dy, r.dz, qx, qy, qz) * inv;
    t = dot3(c.x, c.y, c.z, qx, qy, qz) * inv;
    return det != 0.0f && u >= 0.0f && u <= 1.0f && v >= 0.0f && u + v <= 1.0f &&
           t > r.tmin && t < r.tmax;
}

// -------------------------------------------------------------------------
// traversal stack: kLds entries per lane in LDS, deeper entries spill to a
// per-ray slice of global memory (so the per-ray visit order never depends
// on the stack capacity)
// -------------------------------------------------------------------------
template <int kLds, int kBlock>
struct trav_stack {
    uint2 (*lds)[kBlock];  // [kLds][kBlock]
    uint2 *spill;          // [depth - kLds][spill_stride], may be null if never needed
    uint32_t lane, slot, spill_stride;
    int sp = 0;

    __device__ __forceinline__ void push(uint32_t ref, float tn)
    {
        const uint2 e = make_uint2(ref, __float_as_uint(tn));
        if (kLds > 0 && sp < kLds)
            lds[sp][lane] = e;
        else
            spill[size_t(sp - kLds) * spill_stride + slot] = e;
        ++sp;
    }
    // Pops entries until one with tn <= tmax; returns false when empty.
    __device__ __forceinline__ bool pop(float tmax, uint32_t &ref)
    {
        while (sp > 0) {
            --sp;
            const uint2 e = (kLds > 0 && sp < kLds) ? lds[sp][lane]
                                                     : spill[size_t(sp - kLds) * spill_stride + slot];
            if (!(__uint_as_float(e.y) > tmax)) {
                ref = e.x;
                return true;
            }
        }
        return false;
    }
};

struct scene_view {
    const float4 *nodes;  // 4 float4 per inner node
    const float4 *tris;   // 3 float4 per triangle record
    float root_lo[3], root_hi[3];
    uint32_t root_ref;
    uint32_t n_tris;
};

struct trace_result {
    float t, u, v;
    uint32_t prim;
};

// One ray through the BVH (Algorithm 1: while the ray is alive, descend inner
// nodes, then test the primitives of the leaf reached).  kAny stops at the
// first accepted hit; otherwise the nearest accepted hit is kept.
template <bool kAny, class Isect, class Stack>
__device__ __forceinline__ trace_result traverse(const scene_view &sc, ray_state r, Isect &isect,
                                                 Stack &stack)
{
    trace_result res{__builtin_huge_valf(), 0.0f, 0.0f, kMissPrim};
    if (sc.n_tris == 0) return res;

    float tn;
    isect.on_box_test();
    bool alive = slab(r, sc.root_lo[0], sc.root_lo[1], sc.root_lo[2], sc.root_hi[0],
                      sc.root_hi[1], sc.root_hi[2], tn);
    uint32_t cur = sc.root_ref;

    while (alive) {
        // inner nodes
        while (ref_count(cur) == 0) {
            const float4 *nd = sc.nodes + 4 * size_t(cur);
            const float4 n0 = nd[0], n1 = nd[1], n2 = nd[2];
            const uint4 n3 = *reinterpret_cast<const uint4 *>(nd + 3);
            float tl, tr;
            isect.on_box_test();
            isect.on_box_test();
            const bool hl = slab(r, n0.x, n0.y, n0.z, n0.w, n1.x, n1.y, tl);
            const bool hr = slab(r, n1.z, n1.w, n2.x, n2.y, n2.z, n2.w, tr);
            if (hl && hr) {
                const bool right_first = tr < tl;
                cur = right_first ? n3.y : n3.x;
                stack.push(right_first ? n3.x : n3.y, right_first ? tl : tr);
            } else if (hl) {
                cur = n3.x;
            } else if (hr) {
                cur = n3.y;
            } else if (!stack.pop(r.tmax, cur)) {
                alive = false;
                break;
            }
        }
        if (!alive) break;

        // leaf: its triangles in stored order
        const uint32_t first = ref_index(cur), count = ref_count(cur);
        for (uint32_t j = first; j < first + count; ++j) {
            const float4 *tp = sc.tris + 3 * size_t(j);
            const float4 a = tp[0], b = tp[1], c = tp[2];
            isect.on_tri_test();
            float t, u, v;
            if (triangle(r, a, b, c, t, u, v)) {
                bool ok = true;
                if constexpr (Isect::kFilters)
                    ok = isect.accept(hit_candidate{__float_as_uint(a.w), __float_as_uint(b.w), t, u, v});
                if (ok) {
                    res.t = t;
                    res.u = u;
                    res.v = v;
                    res.prim = __float_as_uint(a.w);
                    if constexpr (kAny) {
                        alive = false;
                        break;
                    } else {
                        r.tmax = t;
                    }
                }
            }
        }
        if (!alive) break;
        alive = stack.pop(r.tmax, cur);
    }
    return res;
}

}  // namespace rtx
