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
//                                      accept call entirely (an intersector
//                                      without a decision adds no work,
//                                      Section 1)
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

#include <type_traits>

#include "rt_batch_layout.hpp"

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
// traversal stack: a ring of kSlots entries per lane in LDS holds the top of
// the stack; when a push would overflow it, the oldest entry moves to a
// per-lane column of global memory, and pops below the ring read it back.
// Every entry survives, so the per-ray visit order never depends on kSlots.
// Entries [0, base) live in global memory, [base, sp) in the ring at slot
// i & (kSlots - 1); at most kSlots - 1 live in the ring, so the slot at sp is
// always free and a push can write it before knowing whether it is kept.
// -------------------------------------------------------------------------
// A pointer into global memory (address space 1).  Typing the spill column
// this way keeps the compiler from merging its accesses with the LDS ring's
// into generic (flat) accesses.
template <class T>
using global_ptr = __attribute__((address_space(1))) T *;

template <int kSlots, int kBlock>
struct ring_stack {
    static_assert((kSlots & (kSlots - 1)) == 0 && kSlots >= 2, "kSlots: power of two >= 2");
    static constexpr uint32_t kMask = kSlots - 1;
    uint2 (*ring)[kBlock];  // [kSlots][kBlock] in LDS
    global_ptr<uint64_t> spill;  // this lane's column: entry i at spill[i * stride]
    uint32_t tid, stride;
    uint32_t sp = 0, base = 0;
    uint32_t floor = 0;  // pops stop here (a nested traversal owns [floor, sp))

    __device__ __forceinline__ void reset()
    {
        sp = 0;
        base = 0;
        floor = 0;
    }

    // Writes e into the free slot; keeps it iff `keep`.
    __device__ __forceinline__ void push_if(bool keep, uint2 e)
    {
        ring[sp & kMask][tid] = e;
        if (keep) {
            ++sp;
            if (sp - base == kSlots) {  // ring full: evict the oldest entry
                spill_store(base, ring[base & kMask][tid]);
                ++base;
            }
        }
    }

    // Pops until an entry with tn <= tmax appears; false when empty.
    __device__ __forceinline__ bool pop(float tmax, uint32_t &ref)
    {
        while (sp > floor) {
            --sp;
            uint2 e;
            if (sp >= base) {
                e = ring[sp & kMask][tid];
            } else {
                e = spill_load(sp);
                base = sp;
            }
            if (!(__uint_as_float(e.y) > tmax)) {
                ref = e.x;
                return true;
            }
        }
        return false;
    }

    __device__ __forceinline__ void spill_store(uint32_t i, uint2 e)
    {
        spill[size_t(i) * stride] = uint64_t(e.x) | (uint64_t(e.y) << 32);
    }
    __device__ __forceinline__ uint2 spill_load(uint32_t i) const
    {
        const uint64_t v = spill[size_t(i) * stride];
        return make_uint2(uint32_t(v), uint32_t(v >> 32));
    }
};

struct scene_view {
    const float4 *nodes;  // 4 float4 per inner node (2 with RT_LAYOUT_Q8, 3 with RT_LAYOUT_F32P,
                          // 8 with RT_LAYOUT_WIDE4)
    const float4 *tris;   // 3 float4 per triangle record
    float root_lo[3], root_hi[3];
    uint32_t root_ref;
    uint32_t n_tris;
    uint32_t layout;      // RT_LAYOUT_F32, RT_LAYOUT_Q8, RT_LAYOUT_F32P or RT_LAYOUT_WIDE4
};

// A child reference of a RT_LAYOUT_F32P node: byte k is the low byte of the
// bit pattern of the child's k-th box word (lo.x, lo.y, lo.z, hi.x).
// Two byte permutes and a shift-or: v_perm_b32 picks each result byte from
// the eight bytes of its operand pair (selector 0-3: the second operand's
// bytes, 4-7: the first's, 0x0c: zero), so perm(b, a, 0x0c0c0400) is
// (a0, b0, 0, 0) -- three instructions where the masks and shifts take six.
__device__ __forceinline__ uint32_t packed_ref(float a, float b, float c, float d)
{
    const uint32_t lo = __builtin_amdgcn_perm(__float_as_uint(b), __float_as_uint(a), 0x0c0c0400u);
    const uint32_t hi = __builtin_amdgcn_perm(__float_as_uint(d), __float_as_uint(c), 0x0c0c0400u);
    return lo | hi << 16;
}

// The two child boxes (lo0, hi0, lo1, hi1) and references of inner node
// `cur`.  RT_LAYOUT_Q8: per axis a, origin = frame word with its low byte
// cleared and scale = 2^(low byte - 127) (both as bit patterns), and each
// 8-bit coordinate q decodes to fma(q, scale, origin).  RT_LAYOUT_F32P: the
// stored words are the boxes as they are, and the references are gathered
// from their low bytes.  The layout is a compile-time choice: a run-time
// branch here merges the paths' loads and costs the float32 layout 6-13 %.
template <uint32_t kLayout>
__device__ __forceinline__ void node_children(const scene_view &sc, uint32_t cur, float (&b)[12],
                                              uint32_t &ref0, uint32_t &ref1)
{
    if constexpr (kLayout == RT_LAYOUT_F32P) {
        const float4 *nd = sc.nodes + 3 * size_t(cur);
        const float4 n0 = nd[0], n1 = nd[1], n2 = nd[2];
        b[0] = n0.x; b[1] = n0.y; b[2] = n0.z; b[3] = n0.w;
        b[4] = n1.x; b[5] = n1.y; b[6] = n1.z; b[7] = n1.w;
        b[8] = n2.x; b[9] = n2.y; b[10] = n2.z; b[11] = n2.w;
        ref0 = packed_ref(b[0], b[1], b[2], b[3]);
        ref1 = packed_ref(b[6], b[7], b[8], b[9]);
    } else if constexpr (kLayout == RT_LAYOUT_Q8) {
        const uint4 *nd = reinterpret_cast<const uint4 *>(sc.nodes) + 2 * size_t(cur);
        const uint4 w0 = nd[0], w1 = nd[1];
        const uint32_t frame[3] = {w0.x, w0.y, w0.z};
        const uint32_t qw[3] = {w0.w, w1.x, w1.y};
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const uint32_t f = frame[k % 3];
            const float q = float((qw[k / 4] >> (8 * (k % 4))) & 0xFFu);
            b[k] = fmaf(q, __uint_as_float((f & 0xFFu) << 23), __uint_as_float(f & ~0xFFu));
        }
        ref0 = w1.z;
        ref1 = w1.w;
    } else {
        const float4 *nd = sc.nodes + 4 * size_t(cur);
        const float4 n0 = nd[0], n1 = nd[1], n2 = nd[2];
        const uint4 n3 = *reinterpret_cast<const uint4 *>(nd + 3);
        b[0] = n0.x; b[1] = n0.y; b[2] = n0.z; b[3] = n0.w;
        b[4] = n1.x; b[5] = n1.y; b[6] = n1.z; b[7] = n1.w;
        b[8] = n2.x; b[9] = n2.y; b[10] = n2.z; b[11] = n2.w;
        ref0 = n3.x;
        ref1 = n3.y;
    }
}

// Order key of a four-wide child: hit children by (tn, child index), every
// missed child after them.  The float's bit pattern is mapped to an unsigned
// integer of the same order (negative values reversed), so one 64-bit
// compare orders the pair.
__device__ __forceinline__ uint64_t wide_key(bool hit, float tn, uint32_t c)
{
    const uint32_t b = __float_as_uint(tn);
    const uint32_t ord = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return hit ? (uint64_t(ord) << 2 | c) : ~uint64_t(0);
}

__device__ __forceinline__ float wide_key_tn(uint64_t k)
{
    const uint32_t ord = uint32_t(k >> 2);
    return __uint_as_float((ord & 0x80000000u) ? (ord & 0x7FFFFFFFu) : ~ord);
}

__device__ __forceinline__ void order2(uint64_t &a, uint64_t &b)
{
    const uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
    a = lo;
    b = hi;
}

// One step at a four-wide node (RT_LAYOUT_WIDE4, 128-B record: lo.x[4],
// hi.x[4], lo.y[4], hi.y[4], lo.z[4], hi.z[4], ref[4]): box-test every used
// child slot, visit the nearest hit child (ties -> the lower slot) and push
// the other hit ones from the farthest to the second nearest; with none hit,
// pop.  The four keys are ordered by a five-comparator sorting network.
template <class Isect, class Stack>
__device__ __forceinline__ bool inner_step_wide(const scene_view &sc, const ray_state &r,
                                                Isect &isect, Stack &st, uint32_t &cur)
{
    const float4 *nd = sc.nodes + 8 * size_t(cur);
    const uint4 rf = *reinterpret_cast<const uint4 *>(nd + 6);
    const float4 lx = nd[0], hx = nd[1], ly = nd[2], hy = nd[3], lz = nd[4], hz = nd[5];
    // all seven fetches in flight before any use: without this fence the
    // scheduler issues the reference word only after the six box words have
    // arrived, a second memory round trip per node
    __builtin_amdgcn_sched_barrier(0);
    const float alx[4] = {lx.x, lx.y, lx.z, lx.w}, ahx[4] = {hx.x, hx.y, hx.z, hx.w};
    const float aly[4] = {ly.x, ly.y, ly.z, ly.w}, ahy[4] = {hy.x, hy.y, hy.z, hy.w};
    const float alz[4] = {lz.x, lz.y, lz.z, lz.w}, ahz[4] = {hz.x, hz.y, hz.z, hz.w};
    const uint32_t ref[4] = {rf.x, rf.y, rf.z, rf.w};
    uint64_t k[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const bool used = ref[c] != RT_WIDE_EMPTY_REF;
        if (used) isect.on_box_test();
        float tn;
        const bool hit = slab(r, alx[c], aly[c], alz[c], ahx[c], ahy[c], ahz[c], tn);
        k[c] = wide_key(used && hit, tn, uint32_t(c));
    }
    order2(k[0], k[1]);
    order2(k[2], k[3]);
    order2(k[0], k[2]);
    order2(k[1], k[3]);
    order2(k[1], k[2]);
    const uint64_t none = ~uint64_t(0);
    // the reference of the key's child slot, by selects rather than branches
    auto ref_of = [&](uint64_t key) {
        const uint32_t c = uint32_t(key);
        const uint32_t r01 = (c & 1u) ? ref[1] : ref[0];
        const uint32_t r23 = (c & 1u) ? ref[3] : ref[2];
        return (c & 2u) ? r23 : r01;
    };
    st.push_if(k[3] != none, make_uint2(ref_of(k[3]), __float_as_uint(wide_key_tn(k[3]))));
    st.push_if(k[2] != none, make_uint2(ref_of(k[2]), __float_as_uint(wide_key_tn(k[2]))));
    st.push_if(k[1] != none, make_uint2(ref_of(k[1]), __float_as_uint(wide_key_tn(k[1]))));
    if (k[0] != none) {
        cur = ref_of(k[0]);
        return true;
    }
    return st.pop(r.tmax, cur);
}

// One inner-node step: test both children's boxes; visit the nearer hit
// child (ties -> child 0) and push the other if both are hit; with neither
// hit, pop.  Returns false when the stack ran empty (ray finished).
template <uint32_t kLayout = RT_LAYOUT_F32, class Isect, class Stack>
__device__ __forceinline__ bool inner_step(const scene_view &sc, const ray_state &r, Isect &isect,
                                           Stack &st, uint32_t &cur)
{
    if constexpr (kLayout == RT_LAYOUT_WIDE4) return inner_step_wide(sc, r, isect, st, cur);
    float b[12];
    uint32_t ref0, ref1;
    node_children<kLayout>(sc, cur, b, ref0, ref1);
    float tl, tr;
    isect.on_box_test();
    isect.on_box_test();
    const bool hl = slab(r, b[0], b[1], b[2], b[3], b[4], b[5], tl);
    const bool hr = slab(r, b[6], b[7], b[8], b[9], b[10], b[11], tr);
    const bool right_first = tr < tl;
    const uint32_t near = (hl && !(hr && right_first)) ? ref0 : ref1;
    const uint32_t far = right_first ? ref0 : ref1;
    const float far_tn = right_first ? tl : tr;
    st.push_if(hl && hr, make_uint2(far, __float_as_uint(far_tn)));
    if (hl || hr) {
        cur = near;
        return true;
    }
    return st.pop(r.tmax, cur);
}

// Result policies: what a query keeps of the accepted hits (Section 3.1).
// commit() receives every accepted candidate in traversal order, may shrink
// the search interval r.tmax, and returns true when the ray is finished.
struct closest_result {  // the nearest accepted hit
    float t, u, v;
    uint32_t prim;
    __device__ __forceinline__ void reset(const ray_state &, uint32_t)
    {
        t = __builtin_huge_valf();
        u = v = 0.0f;
        prim = kMissPrim;
    }
    __device__ __forceinline__ bool commit(ray_state &r, float tt, float uu, float vv, uint32_t p,
                                           uint32_t)
    {
        t = tt;
        u = uu;
        v = vv;
        prim = p;
        r.tmax = tt;
        return false;
    }
};

struct any_result {  // the first accepted hit met
    uint32_t prim;
    __device__ __forceinline__ void reset(const ray_state &, uint32_t) { prim = kMissPrim; }
    __device__ __forceinline__ bool commit(ray_state &, float, float, float, uint32_t p, uint32_t)
    {
        prim = p;
        return true;
    }
};

// The k nearest accepted hits (k <= kMax, a run-time value), sorted by t;
// a new hit goes after every kept hit with the same t.  Once k hits are kept,
// the k-th distance bounds the search.  The list lives in registers as
// (t, triangle record index) pairs only -- every loop over it is unrolled, so
// no index is dynamic -- and the barycentrics of the kept hits are recomputed
// from their records when the ray is written (the same float32 operations on
// the same ray give the same u, v), which halves the list's registers.
template <int kMax>
struct multi_result {
    float t[kMax];
    uint32_t rec[kMax];
    uint32_t n, k;
    float tmax0;
    __device__ __forceinline__ void reset(const ray_state &r, uint32_t kk)
    {
#pragma unroll
        for (int i = 0; i < kMax; ++i) {
            t[i] = __builtin_huge_valf();
            rec[i] = kMissPrim;
        }
        n = 0;
        k = kk;
        tmax0 = r.tmax;
    }
    __device__ __forceinline__ bool commit(ray_state &r, float tt, float, float, uint32_t,
                                           uint32_t j)
    {
        // the new hit goes into the first slot whose kept hit is strictly
        // farther; from there on every kept hit moves down one slot (a plain
        // shift, so kept hits of equal t keep their order); what falls off
        // slot k-1 is dropped
        float ct = tt;
        uint32_t cj = j;
        float tk = __builtin_huge_valf();
        bool shifting = false;
#pragma unroll
        for (int i = 0; i < kMax; ++i) {
            const bool live = uint32_t(i) < k;
            const bool take = live && (shifting || ct < t[i]);
            shifting = take;
            const float st = t[i];
            const uint32_t sj = rec[i];
            t[i] = take ? ct : st;
            rec[i] = take ? cj : sj;
            ct = take ? st : ct;
            cj = take ? sj : cj;
            if (uint32_t(i) + 1 == k) tk = t[i];
        }
        n = n < k ? n + 1 : k;
        r.tmax = fminf(tmax0, tk);
        return false;
    }
};

// The triangles of one leaf, in stored order.  Returns true iff the result
// policy finished the ray.
template <class Result, class Isect>
__device__ __forceinline__ bool leaf_step(const scene_view &sc, ray_state &r, Isect &isect,
                                          uint32_t ref, Result &res)
{
    const uint32_t first = ref_index(ref), count = ref_count(ref);
    for (uint32_t j = first; j < first + count; ++j) {
        const float4 *tp = sc.tris + 3 * size_t(j);
        const float4 a = tp[0], b = tp[1], c = tp[2];
        isect.on_tri_test();
        float t, u, v;
        if (triangle(r, a, b, c, t, u, v)) {
            bool ok = true;
            if constexpr (Isect::kFilters)
                ok = isect.accept(hit_candidate{__float_as_uint(a.w), __float_as_uint(b.w), t, u, v});
            if (ok && res.commit(r, t, u, v, __float_as_uint(a.w), j)) return true;
        }
    }
    return false;
}

// Root test of a fresh ray: false if the ray misses the scene (or the scene
// is empty), in which case it is finished with a miss.
template <class Isect>
__device__ __forceinline__ bool root_step(const scene_view &sc, const ray_state &r, Isect &isect)
{
    if (sc.n_tris == 0) return false;
    float tn;
    isect.on_box_test();
    return slab(r, sc.root_lo[0], sc.root_lo[1], sc.root_lo[2], sc.root_hi[0], sc.root_hi[1],
                sc.root_hi[2], tn);
}

// Index of the scene whose ray range holds ray `id` (binary search over the
// ray_begin prefix; empty scenes are skipped naturally).
__device__ __forceinline__ uint32_t batch_scene_of(const uint32_t *prefix, uint32_t n_scenes,
                                                   uint32_t id)
{
    uint32_t lo = 0, hi = n_scenes;  // invariant: prefix[lo] <= id < prefix[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (prefix[mid] <= id)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// -------------------------------------------------------------------------
// the traversal kernel
// -------------------------------------------------------------------------
struct kernel_args {
    scene_view sc;
    const float4 *rays;  // 2 float4 per ray
    uint32_t n_rays;
    void *out;           // float4 hits (closest, [n][k] for multi) or uint32 occluders (any)
    uint32_t *n_hits;    // multi-hit: kept hits per ray
    uint32_t multi_k;    // multi-hit: hits kept per ray
    uint4 *counters;
    const unsigned char *batch;  // batched launch: the scene table (else null)
    uint64_t *spill;     // [spill entries][gridDim.x * kBlock]
    uint32_t *queue;     // kQueueHeads work-queue heads, kQueueStride apart, zero at launch
    uint32_t tile_w8;    // tiled schedule: image width / 8 (0: rays in index order)
    uint32_t tiled;      // rays [0, tiled) are whole rows of 8 x 8 tiles
    const uint32_t *order;  // longest-path-first: chunk to take at each position (else null)
};

// The ray a lane takes for schedule position `pos`: in a tiled schedule,
// position 64 c + j of the first `tiled` rays is pixel j (row-major) of
// tile c, tiles numbered row-major over an image a.tile_w8 tiles wide.
__device__ __forceinline__ uint32_t scheduled_ray(const kernel_args &a, uint32_t pos)
{
    if (a.tile_w8 == 0 || pos >= a.tiled) return pos;
    const uint32_t c = pos >> 6, j = pos & 63u;
    const uint32_t ty = c / a.tile_w8, tx = c - ty * a.tile_w8;
    return ((ty << 3) + (j >> 3)) * (a.tile_w8 << 3) + (tx << 3) + (j & 7u);
}

// Work-queue heads of a persistent launch: one per XCD (MI355X has 8), each
// in its own 128-byte cache line.
constexpr uint32_t kQueueHeads = 8;
constexpr uint32_t kQueueStride = 32;  // uint32 words

// Rays are handed to lanes, not to waves: a wave takes kChunk consecutive rays
// at a time -- from its own static slice (kQueue = false: wave w owns rays
// [w kChunk, (w+1) kChunk)) or from a global atomic queue shared by a grid of
// kPersistentWaves resident waves (kQueue = true) -- and gives the next ray
// of its chunk to any lane whose ray has finished, so that lanes do not idle
// behind the slowest ray of the wave.  Each ray's own traversal (Algorithm 1:
// descend inner nodes, then test the leaf's triangles, until the stack is
// empty) is exactly what it would be alone.
template <class Result>  // closest_result or any_result
__device__ __forceinline__ bool res_hit(const Result &res)
{
    return res.prim != kMissPrim;
}

// Writes ray `ray`'s record(s); sc and r are the lane's scene and ray state
// (the multi-hit list recomputes its barycentrics from them).
template <class Result>
__device__ __forceinline__ void write_result(const kernel_args &a, const scene_view &sc,
                                             const ray_state &r, uint32_t ray, const Result &res)
{
    if constexpr (std::is_same_v<Result, any_result>) {
        static_cast<uint32_t *>(a.out)[ray] = res.prim;
    } else if constexpr (std::is_same_v<Result, closest_result>) {
        static_cast<float4 *>(a.out)[ray] =
            make_float4(res.t, __uint_as_float(res.prim), res.u, res.v);
    } else {
        float4 *o = static_cast<float4 *>(a.out) + size_t(ray) * a.multi_k;
#pragma unroll
        for (int i = 0; i < int(sizeof(res.t) / sizeof(float)); ++i) {
            if (uint32_t(i) >= a.multi_k) continue;
            float4 h = make_float4(__builtin_huge_valf(), __uint_as_float(kMissPrim), 0.0f, 0.0f);
            if (uint32_t(i) < res.n) {
                const float4 *tp = sc.tris + 3 * size_t(res.rec[i]);
                const float4 ta = tp[0], tb = tp[1], tc = tp[2];
                float tt, uu, vv;
                triangle(r, ta, tb, tc, tt, uu, vv);
                h = make_float4(res.t[i], ta.w, uu, vv);
            }
            o[i] = h;
        }
        a.n_hits[ray] = res.n;
    }
}

// Per-ray intersector parameters of a batched launch: the alpha mask takes
// its texture data from the ray's scene record, other intersectors use the
// launch's parameters.
template <class Isect>
__device__ __forceinline__ typename Isect::params batch_params(const typename Isect::params &p,
                                                               const batch_scene &bs)
{
    if constexpr (std::is_base_of_v<alpha_intersector, Isect>) {
        typename Isect::params q = p;
        q.texcoords = bs.texcoords;
        q.textures = bs.textures;
        q.width = bs.tex_width;
        q.height = bs.tex_height;
        q.alpha_min = bs.alpha_min;
        return q;
    } else {
        return p;
    }
}

// The wave's supply of rays: its current chunk [next, end) and, in a queue
// launch, the queue state.  Chunks past the static first ones are dealt
// round-robin to kQueueHeads heads; a wave draws from the head of its block's
// XCD (blocks are dispatched to the XCDs round-robin) and, once that head is
// exhausted, from the others in turn.
template <int kBlock, int kChunk, bool kQueue>
struct ray_feed {
    uint32_t next, end;
    bool drained;  // no further chunk will come
    uint32_t head, dead_heads;

    // The rays of the chunk at schedule position c (the chunk itself, or the
    // one a longest-path-first order puts there).
    __device__ __forceinline__ void set_chunk(uint32_t c, uint32_t n_rays, const uint32_t *order)
    {
        if (order) c = order[c];
        next = c * uint32_t(kChunk);
        end = min(next + uint32_t(kChunk), n_rays);
    }

    __device__ __forceinline__ ray_feed(uint32_t n_rays, uint32_t gtid, const uint32_t *order)
    {
        // every wave's first chunk is static (position = wave index), so a
        // queue launch does not start with every wave on an atomic
        const uint32_t c = gtid / 64;
        if (c * uint64_t(kChunk) < n_rays) {
            set_chunk(c, n_rays, order);
        } else {
            next = end = 0;
        }
        drained = !kQueue;
        head = blockIdx.x % kQueueHeads;
        dead_heads = 0;
    }

    // Wave-wide, with the wave's idle-lane mask: makes sure the chunk holds
    // rays (drawing a new chunk from the queue if needed); false if none are
    // left for now.
    __device__ __forceinline__ bool refill(uint64_t idle, uint32_t n_rays, uint32_t *queue,
                                          const uint32_t *order)
    {
        if constexpr (kQueue) {
            if (idle != 0 && next >= end && !drained) {
                const uint32_t n_chunks = (n_rays + uint32_t(kChunk) - 1) / uint32_t(kChunk);
                const uint32_t first_dynamic = gridDim.x * (uint32_t(kBlock) / 64);
                while (dead_heads != (1u << kQueueHeads) - 1) {
                    uint32_t k = 0;
                    if (__lane_id() == 0) k = atomicAdd(queue + head * kQueueStride, 1u);
                    k = __builtin_amdgcn_readfirstlane(k);
                    const uint64_t chunk = uint64_t(first_dynamic) + head + uint64_t(kQueueHeads) * k;
                    if (chunk < n_chunks) {
                        set_chunk(uint32_t(chunk), n_rays, order);
                        break;
                    }
                    dead_heads |= 1u << head;
                    head = (head + 1) % kQueueHeads;
                }
                drained = dead_heads == (1u << kQueueHeads) - 1;
            }
        }
        return idle != 0 && next < end;
    }

    // Wave-wide after a successful refill: the idle lanes take the next rays
    // in lane order; a lane's ray id is valid iff it is below `end` (read
    // before the call).
    __device__ __forceinline__ uint32_t take(uint64_t idle, uint64_t lanes_below)
    {
        const uint32_t id = next + uint32_t(__popcll(idle & lanes_below));
        next = min(next + uint32_t(__popcll(idle)), end);
        return id;
    }

    __device__ __forceinline__ bool exhausted() const { return drained && next >= end; }
};

// A wave leaves its inner-node phase for the leaf phase once fewer than
// kLeafBreak/16 of its busy lanes are still at inner nodes: waiting for the
// last lane to reach a leaf would issue every node fetch for a few lanes.
constexpr uint32_t kLeafBreak = 8;
// Lane masks from compares: an LLVM integer-compare predicate code for
// __builtin_amdgcn_uicmp (ne, unsigned less-than), the first reference of
// a leaf (count 1 << 29: inner references are below it), and the key of a
// finished lane.
constexpr int kIcmpNE = 33, kIcmpULT = 36;
constexpr uint32_t kRefCountUnit = 1u << 29;
constexpr uint32_t kNoRef = 0xFFFFFFFFu;

__device__ __forceinline__ bool leave_inner_phase(uint32_t n_inner, uint32_t n_leaf)
{
    return 16u * n_inner < kLeafBreak * (n_inner + n_leaf);
}

// Waves per SIMD a traversal kernel must fit.  The k <= 4 multi-hit list fits
// 6 (80 VGPRs) without spilling, which measured +2 % (alpha) to +11 %
// (accept-all) over the compiler's 5; the other kernels keep the compiler's
// choice (6 waves spill the k <= 8 list: -15 %).
template <class Result>
struct min_waves_per_simd {
    static constexpr int value = 1;
};
template <>
struct min_waves_per_simd<multi_result<4>> {
    static constexpr int value = 6;
};

template <class Isect, class Result, int kSlots, int kBlock, int kChunk, bool kQueue,
          bool kBatched = false, uint32_t kLayout = RT_LAYOUT_F32>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(min_waves_per_simd<Result>::value)))
void trace_kernel(kernel_args a, typename Isect::params p)
{
    static_assert(kBlock % 64 == 0 && kChunk % 32 == 0, "wave64 shapes");
    __shared__ uint2 ring[kSlots][kBlock];
    const uint32_t tid = threadIdx.x;
    const uint32_t gtid = blockIdx.x * kBlock + tid;
    const uint32_t lane = __lane_id();
    const uint64_t lanes_below = (uint64_t(1) << lane) - 1;

    ray_feed<kBlock, kChunk, kQueue> feed(a.n_rays, gtid, a.order);

    ring_stack<kSlots, kBlock> st{ring, (global_ptr<uint64_t>)(a.spill + gtid), tid,
                                  gridDim.x * uint32_t(kBlock)};
    bool active = false;
    uint32_t ray_id = 0, cur = 0;
    ray_state r{};
    scene_view sc = a.sc;  // per lane in a batched launch
    Isect isect(p);
    Result res;
    res.reset(r, a.multi_k);

    auto finish = [&]() {
        write_result(a, sc, r, ray_id, res);
        if constexpr (Isect::kCounts)
            a.counters[ray_id] = make_uint4(isect.num_boxes, isect.num_tris, isect.num_candidates,
                                            isect.num_accepted);
    };

    for (;;) {
        const uint64_t idle = __ballot(!active);
        if (feed.refill(idle, a.n_rays, a.queue, a.order)) {
            const uint32_t id = feed.take(idle, lanes_below);
            if (!active && id < feed.end) {
                ray_id = scheduled_ray(a, id);
                r = make_ray(a.rays[2 * size_t(ray_id)], a.rays[2 * size_t(ray_id) + 1]);
                if constexpr (kBatched) {
                    const uint32_t n_scenes = *reinterpret_cast<const uint32_t *>(a.batch);
                    const uint32_t *prefix =
                        reinterpret_cast<const uint32_t *>(a.batch + batch_prefix_offset());
                    const batch_scene &bs = reinterpret_cast<const batch_scene *>(
                        a.batch + batch_records_offset(n_scenes))[batch_scene_of(prefix, n_scenes, id)];
                    sc.nodes = bs.nodes;
                    sc.tris = bs.tris;
                    sc.root_lo[0] = bs.root_lo[0];
                    sc.root_lo[1] = bs.root_lo[1];
                    sc.root_lo[2] = bs.root_lo[2];
                    sc.root_hi[0] = bs.root_hi[0];
                    sc.root_hi[1] = bs.root_hi[1];
                    sc.root_hi[2] = bs.root_hi[2];
                    sc.root_ref = bs.root_ref;
                    sc.n_tris = bs.n_tris;
                    sc.layout = bs.layout;
                    isect = Isect(batch_params<Isect>(p, bs));
                } else {
                    isect = Isect(p);
                }
                st.reset();
                res.reset(r, a.multi_k);
                cur = sc.root_ref;
                active = root_step(sc, r, isect);
                if (!active) finish();
            }
        }
        if (__ballot(active) == 0) {
            if (feed.exhausted()) break;
            continue;
        }
        if (active) {
            // inner phase: lanes at inner nodes step on while enough of them
            // remain; lanes already at a leaf wait (their ray's order is
            // unchanged -- a lane that leaves this phase at an inner node
            // simply continues from it in the next round).  The wave runs
            // this phase at raised issue priority and its leaf phase at the
            // lowest: on a SIMD shared by waves in both phases, node fetches
            // then issue ahead of the longer dependent leaf chains (measured
            // +2.6 % alpha billboards, +1.8 % spheres, default unchanged)
            __builtin_amdgcn_s_setprio(1);
            for (;;) {
                // the two lane masks straight from compares (a ballot of a
                // combined condition costs a select and a compare more
                // each): finished lanes carry the key kNoRef, which no
                // reference equals (a leaf of 7 triangles at index 2^29 - 1
                // would end past the largest triangle count)
                const uint32_t key = active ? cur : kNoRef;
                const uint64_t mi = __builtin_amdgcn_uicmp(key, kRefCountUnit, kIcmpULT);
                if (mi == 0) break;
                const uint64_t ml = __builtin_amdgcn_uicmp(key, kNoRef, kIcmpNE) & ~mi;
                const bool in_inner = key < kRefCountUnit;
                if (ml != 0 && leave_inner_phase(uint32_t(__popcll(mi)), uint32_t(__popcll(ml))))
                    break;
                if (in_inner && !inner_step<kLayout>(sc, r, isect, st, cur)) active = false;
            }
            __builtin_amdgcn_s_setprio(0);
            if (active && ref_count(cur) != 0) {
                if (leaf_step(sc, r, isect, cur, res))
                    active = false;
                else
                    active = st.pop(r.tmax, cur);
            }
            if (!active) finish();
        }
    }
}

// -------------------------------------------------------------------------
// instancing (Section 3.2: BVHs as primitives of a top-level BVH)
// -------------------------------------------------------------------------
// World ray -> object ray of an instance with object_from_world map m
// (row-major 3x4); t and the barycentrics of a hit are unchanged.
__device__ __forceinline__ ray_state object_ray(const ray_state &w, const float m[12])
{
    float4 o, d;
    o.x = fmaf(m[0], w.ox, fmaf(m[1], w.oy, fmaf(m[2], w.oz, m[3])));
    o.y = fmaf(m[4], w.ox, fmaf(m[5], w.oy, fmaf(m[6], w.oz, m[7])));
    o.z = fmaf(m[8], w.ox, fmaf(m[9], w.oy, fmaf(m[10], w.oz, m[11])));
    o.w = w.tmin;
    d.x = fmaf(m[0], w.dx, fmaf(m[1], w.dy, m[2] * w.dz));
    d.y = fmaf(m[4], w.dx, fmaf(m[5], w.dy, m[6] * w.dz));
    d.z = fmaf(m[8], w.dx, fmaf(m[9], w.dy, m[10] * w.dz));
    d.w = w.tmax;
    return make_ray(o, d);
}

// One ray per lane.  The top-level BVH (built over the instances' world
// boxes; its leaf records carry instance indices) is walked like any BVH; at
// a top-level leaf each instance in stored order is entered by a full
// traversal of its bottom-level BVH with the object ray, on the same stack
// above a floor, sharing the distance bound; then the top level resumes.
template <class Isect, class Result, int kSlots>
__global__ __launch_bounds__(64) void trace_instanced_kernel(kernel_args a, const unsigned char *table,
                                                             uint32_t *inst_out,
                                                             typename Isect::params p)
{
    __shared__ uint2 ring[kSlots][64];
    const uint32_t tid = threadIdx.x;
    const uint32_t pos = blockIdx.x * 64 + tid;
    if (pos >= a.n_rays) return;
    const uint32_t i = scheduled_ray(a, pos);  // tiled schedule, else pos
    ring_stack<kSlots, 64> st{ring, (global_ptr<uint64_t>)(a.spill + pos), tid, gridDim.x * 64u};
    ray_state rw = make_ray(a.rays[2 * size_t(i)], a.rays[2 * size_t(i) + 1]);
    Isect isect(p);
    Result res;
    res.reset(rw, 1);
    uint32_t inst_hit = kMissPrim;
    const uint32_t n_blas = reinterpret_cast<const uint32_t *>(table)[0];
    const uint32_t n_inst = reinterpret_cast<const uint32_t *>(table)[1];
    const blas_record *blas = reinterpret_cast<const blas_record *>(table + instance_blas_offset());
    const instance_record *inst =
        reinterpret_cast<const instance_record *>(table + instance_records_offset(n_blas));
    const scene_view &tl = a.sc;
    bool done = false;
    uint32_t cur = tl.root_ref;
    bool alive = root_step(tl, rw, isect);
    while (alive && !done) {
        while (ref_count(cur) == 0) {
            if (!inner_step(tl, rw, isect, st, cur)) {
                alive = false;
                break;
            }
        }
        if (!alive) break;
        const uint32_t first = ref_index(cur), count = ref_count(cur);
        for (uint32_t j = first; j < first + count && !done; ++j) {
            const uint32_t q = __float_as_uint(tl.tris[3 * size_t(j)].w);
            if (q >= n_inst) continue;
            const instance_record &ir = inst[q];
            const uint32_t b = ir.blas;
            if (b >= n_blas) continue;
            float m[12];
#pragma unroll
            for (int k = 0; k < 12; ++k) m[k] = ir.m[k];
            ray_state ro = object_ray(rw, m);
            const blas_record &br = blas[b];
            scene_view bv;
            bv.nodes = br.nodes;
            bv.tris = br.tris;
            bv.root_lo[0] = br.root_lo[0];
            bv.root_lo[1] = br.root_lo[1];
            bv.root_lo[2] = br.root_lo[2];
            bv.root_hi[0] = br.root_hi[0];
            bv.root_hi[1] = br.root_hi[1];
            bv.root_hi[2] = br.root_hi[2];
            bv.root_ref = br.root_ref;
            bv.n_tris = br.n_tris;
            bv.layout = br.layout;
            // the alpha mask reads the texture coordinates of the entered mesh
            if constexpr (std::is_base_of_v<alpha_intersector, Isect>) isect.p.texcoords = br.texcoords;
            const float t_before = ro.tmax;
            st.floor = st.sp;
            if (root_step(bv, ro, isect)) {
                uint32_t c2 = bv.root_ref;
                bool alive2 = true;
                while (alive2) {
                    while (ref_count(c2) == 0) {
                        if (!inner_step(bv, ro, isect, st, c2)) {
                            alive2 = false;
                            break;
                        }
                    }
                    if (!alive2) break;
                    if (leaf_step(bv, ro, isect, c2, res)) {
                        done = true;
                        break;
                    }
                    alive2 = st.pop(ro.tmax, c2);
                }
            }
            st.floor = 0;
            if (done || ro.tmax != t_before) inst_hit = q;
            rw.tmax = ro.tmax;
        }
        if (done) break;
        alive = st.pop(rw.tmax, cur);
    }
    write_result(a, tl, rw, i, res);
    if (inst_out) inst_out[i] = res_hit(res) ? inst_hit : kMissPrim;
    if constexpr (Isect::kCounts)
        a.counters[i] = make_uint4(isect.num_boxes, isect.num_tris, isect.num_candidates,
                                   isect.num_accepted);
}

// Zeroes the work-queue heads before a kQueue launch (a kernel rather than a
// memset, so that the pair can be captured in a graph).
static __global__ void reset_queue_kernel(uint32_t *queue)
{
    if (threadIdx.x < kQueueHeads) queue[threadIdx.x * kQueueStride] = 0;
}

// -------------------------------------------------------------------------
// longest-path-first chunk order (two small kernels before the traversal)
// area: keys[n_chunks], order[n_chunks], then one row of kOrderBuckets
// per-block tallies for each block of the keying kernel
// -------------------------------------------------------------------------
constexpr uint32_t kOrderKeysBlock = 1024;
constexpr uint32_t kOrderSamples = 4;
constexpr uint32_t kOrderRowChunks = kOrderKeysBlock / kOrderSamples;  // chunks per block
constexpr uint32_t kOrderBuckets = 64;

// Four lanes per chunk: the chunk's key is 63 minus the bucket (64 steps of
// the scene box's diagonal) of the longest interval stretch inside the box
// among four of its rays, the ends of its first and last runs of 8 (the
// corners of an 8 x 8 tile), so that sorting keys ascending puts long chunks
// first.  Block b writes its chunks' keys and, in row b of the tallies, how
// many of them fall in each bucket (every row is written whole, so the area
// needs no clearing beforehand).
static __global__ __launch_bounds__(kOrderKeysBlock) void order_keys_kernel(
    kernel_args a, uint32_t chunk, uint32_t n_chunks, float buckets_per_length, uint32_t *keys,
    uint32_t *tallies)
{
    __shared__ uint32_t tally[kOrderBuckets];
    if (threadIdx.x < kOrderBuckets) tally[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t c = (blockIdx.x * blockDim.x + threadIdx.x) / kOrderSamples;
    const uint32_t sample = threadIdx.x % kOrderSamples;
    // 0, 7, chunk - 8, chunk - 1 (chunks are multiples of 32 rays)
    const uint32_t j = (sample & 2u ? chunk - 8u : 0u) + (sample & 1u ? 7u : 0u);
    float len = 0.0f;
    const uint32_t pos = c * chunk + j;
    if (c < n_chunks && pos < a.n_rays) {
        const uint32_t id = scheduled_ray(a, pos);
        const ray_state r = make_ray(a.rays[2 * size_t(id)], a.rays[2 * size_t(id) + 1]);
        float tn;
        if (slab(r, a.sc.root_lo[0], a.sc.root_lo[1], a.sc.root_lo[2], a.sc.root_hi[0],
                 a.sc.root_hi[1], a.sc.root_hi[2], tn)) {
            const float tf = fminf(fminf(fminf(fmaxf(fmaf(a.sc.root_lo[0], r.ix, -r.bx),
                                                     fmaf(a.sc.root_hi[0], r.ix, -r.bx)),
                                               fmaxf(fmaf(a.sc.root_lo[1], r.iy, -r.by),
                                                     fmaf(a.sc.root_hi[1], r.iy, -r.by))),
                                         fmaxf(fmaf(a.sc.root_lo[2], r.iz, -r.bz),
                                               fmaf(a.sc.root_hi[2], r.iz, -r.bz))),
                                   r.tmax);
            len = tf - tn;
        }
    }
    for (uint32_t off = kOrderSamples / 2; off > 0; off >>= 1)
        len = fmaxf(len, __shfl_xor(len, int(off)));
    if (sample == 0 && c < n_chunks) {
        const float q = fminf(len * buckets_per_length, float(kOrderBuckets - 1));
        const uint32_t key = kOrderBuckets - 1 - (q >= 0.0f ? uint32_t(q) : 0u);
        keys[c] = key;
        atomicAdd(tally + key, 1u);
    }
    __syncthreads();
    if (threadIdx.x < kOrderBuckets)
        tallies[blockIdx.x * kOrderBuckets + threadIdx.x] = tally[threadIdx.x];
}

// Scatters the chunk indices into ascending key order; block b takes the
// keying kernel's block b's chunks.  Wave w sums the tally rows w, w + 4, ...
// per bucket (over all rows, and over the rows before b); a bucket's base is
// the exclusive scan of the totals plus the counts of earlier blocks, and a
// chunk's place within its block and bucket comes from an LDS tally.  Block 0
// also zeroes the work-queue heads for the traversal that follows.
constexpr uint32_t kOrderScatterBlock = kOrderRowChunks;
static __global__ __launch_bounds__(kOrderScatterBlock) void order_scatter_kernel(
    uint32_t n_chunks, uint32_t n_rows, const uint32_t *keys, const uint32_t *tallies,
    uint32_t *order, uint32_t *queue)
{
    constexpr uint32_t kWaves = kOrderScatterBlock / 64;
    __shared__ uint32_t total[kWaves][kOrderBuckets], before[kWaves][kOrderBuckets];
    __shared__ uint32_t base[kOrderBuckets], tally[kOrderBuckets];
    const uint32_t t = threadIdx.x, w = t / 64, bucket = t % 64;
    if (blockIdx.x == 0 && queue != nullptr && t < kQueueHeads) queue[t * kQueueStride] = 0;
    uint32_t sum = 0, sum_before = 0;
#pragma unroll 8
    for (uint32_t row = w; row < n_rows; row += kWaves) {
        const uint32_t v = tallies[row * kOrderBuckets + bucket];
        sum += v;
        sum_before += row < blockIdx.x ? v : 0u;
    }
    total[w][bucket] = sum;
    before[w][bucket] = sum_before;
    if (t < kOrderBuckets) tally[t] = 0;
    __syncthreads();
    if (t < kOrderBuckets) {
        uint32_t all = 0, mine = 0;
        for (uint32_t k = 0; k < kWaves; ++k) {
            all += total[k][t];
            mine += before[k][t];
        }
        uint32_t incl = all;  // inclusive scan over the 64 buckets (one wave)
        for (uint32_t off = 1; off < kOrderBuckets; off <<= 1) {
            const uint32_t u = __shfl_up(incl, off);
            if (t >= off) incl += u;
        }
        base[t] = incl - all + mine;
    }
    __syncthreads();
    const uint32_t c = blockIdx.x * kOrderScatterBlock + t;
    if (c < n_chunks) {
        const uint32_t key = keys[c];
        order[base[key] + atomicAdd(tally + key, 1u)] = c;
    }
}

}  // namespace rtx
