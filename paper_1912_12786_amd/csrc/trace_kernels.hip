// Traversal kernels of librtx for gfx950.
//
// One ray per lane (wave64).  Each lane walks the BVH with the while-while
// scheme (Algorithm 1): the wave's lanes that are still descending inner
// nodes run together, then the lanes that reached a leaf test its triangles
// together.  The intersector is a template parameter, so its accept decision
// and counters are inlined into the triangle loop (Section 3.2: the
// intersect calls are replaced at compile time); the default intersector
// compiles to no code.  The traversal stack keeps its top entries in LDS,
// laid out [entry][lane] so that a wave's pushes and pops touch consecutive
// 8-byte words; deeper entries go to a per-ray slice of the caller's
// workspace.
#include <hip/hip_runtime.h>

#include <cmath>

#include "rt_launch.hpp"

namespace rtx {

// -------------------------------------------------------------------------
// Runtime-dispatched intersectors: the same three decisions selected per
// candidate at run time, as a library linked without templates must do
// (Section 1: a runtime check whether a filter was registered, then a call).
// They exist to measure what compile-time injection saves; results are
// bit-identical to the compile-time intersectors.
// -------------------------------------------------------------------------
struct runtime_params {
    alpha_intersector::params alpha;
    uint32_t checker_n;
    uint32_t kind;  // rt_isect_kind
};

// (a) a runtime switch over inlined filter code
struct runtime_switch_intersector : intersector_base {
    static constexpr bool kFilters = true;
    using params = runtime_params;
    runtime_params p;
    __device__ explicit runtime_switch_intersector(const params &pp) : p(pp) {}
    __device__ __forceinline__ bool accept(const hit_candidate &c)
    {
        if (p.kind == RT_ISECT_ALPHA) return alpha_intersector(p.alpha).accept(c);
        if (p.kind == RT_ISECT_PROCEDURAL)
            return checker_intersector(checker_intersector::params{p.checker_n}).accept(c);
        return true;
    }
};

// (b) an indirect call through a table of filter functions
typedef bool (*accept_fn)(hit_candidate, runtime_params);
__device__ __noinline__ bool accept_all_fn(hit_candidate, runtime_params) { return true; }
__device__ __noinline__ bool accept_alpha_fn(hit_candidate c, runtime_params p)
{
    return alpha_intersector(p.alpha).accept(c);
}
__device__ __noinline__ bool accept_checker_fn(hit_candidate c, runtime_params p)
{
    return checker_intersector(checker_intersector::params{p.checker_n}).accept(c);
}
__device__ accept_fn g_accept_table[3] = {accept_all_fn, accept_alpha_fn, accept_checker_fn};

struct runtime_call_intersector : intersector_base {
    static constexpr bool kFilters = true;
    using params = runtime_params;
    runtime_params p;
    __device__ explicit runtime_call_intersector(const params &pp) : p(pp) {}
    __device__ __forceinline__ bool accept(const hit_candidate &c)
    {
        return g_accept_table[p.kind < 3 ? p.kind : 0](c, p);
    }
};

// (block, LDS ring slots, rays per chunk, global queue); the first is the default
const LaunchShape kShapes[] = {kDefaultShape,   {64, 8, 64, 0},   {64, 16, 64, 1}, {256, 8, 64, 1},
                               {128, 8, 64, 1}, {64, 8, 128, 1}, {256, 16, 64, 1},
                               {64, 8, 32, 1}};
const uint32_t kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

namespace {

template <class Isect, int kSlots, int kBlock, int kChunk, bool kQueue, uint32_t kLayout>
rt_status dispatch_query(const TraceRequest &q, const kernel_args &a,
                         const typename Isect::params &p, const char **err)
{
    hipStream_t s = static_cast<hipStream_t>(q.stream);
    if (q.batch) {
        if (q.query != Query::Closest) {
            *err = "batched launches support the closest-hit query only";
            return RT_ERR_UNSUPPORTED;
        }
        return launch_one<Isect, closest_result, kSlots, kBlock, kChunk, kQueue, true, kLayout>(
            a, p, s, err, q.waves_per_simd);
    }
    switch (q.query) {
    case Query::Any:
        return launch_one<Isect, any_result, kSlots, kBlock, kChunk, kQueue, false, kLayout>(
            a, p, s, err, q.waves_per_simd);
    case Query::Multi:
        // the kept list lives in registers: a short list for small k keeps
        // the kernel's register use (and so its occupancy) closer to closest-hit
        if (q.multi_k <= 4)
            return launch_one<Isect, multi_result<4>, kSlots, kBlock, kChunk, kQueue, false,
                              kLayout>(a, p, s, err, q.waves_per_simd);
        return launch_one<Isect, multi_result<RT_MAX_MULTI>, kSlots, kBlock, kChunk, kQueue, false,
                          kLayout>(a, p, s, err, q.waves_per_simd);
    case Query::Closest:
        break;
    }
    return launch_one<Isect, closest_result, kSlots, kBlock, kChunk, kQueue, false, kLayout>(
        a, p, s, err, q.waves_per_simd);
}

template <class Base, int kSlots, int kBlock, int kChunk, bool kQueue, uint32_t kLayout>
rt_status dispatch_count(const TraceRequest &q, const kernel_args &a,
                         const typename Base::params &p, const char **err)
{
    if (q.count)
        return dispatch_query<counting_intersector<Base>, kSlots, kBlock, kChunk, kQueue, kLayout>(
            q, a, p, err);
    return dispatch_query<Base, kSlots, kBlock, kChunk, kQueue, kLayout>(q, a, p, err);
}

template <int kSlots, int kBlock, int kChunk, bool kQueue>
rt_status dispatch_runtime(const TraceRequest &q, const kernel_args &a, const char **err)
{
    runtime_params rp;
    rp.alpha.texcoords = reinterpret_cast<const float2 *>(q.alpha.texcoords);
    rp.alpha.textures = q.alpha.textures;
    rp.alpha.width = q.alpha.width;
    rp.alpha.height = q.alpha.height;
    rp.alpha.alpha_min = q.alpha.alpha_min;
    rp.checker_n = q.checker.checker_n;
    rp.kind = uint32_t(q.kind);
    hipStream_t s = static_cast<hipStream_t>(q.stream);
    if (q.runtime_dispatch == 1)
        return launch_one<runtime_switch_intersector, closest_result, kSlots, kBlock, kChunk, kQueue>(
            a, rp, s, err, q.waves_per_simd);
    return launch_one<runtime_call_intersector, closest_result, kSlots, kBlock, kChunk, kQueue>(
        a, rp, s, err, q.waves_per_simd);
}

template <int kSlots, int kBlock, int kChunk, bool kQueue, uint32_t kLayout = RT_LAYOUT_F32>
rt_status dispatch_kind(const TraceRequest &q, const kernel_args &a, const char **err)
{
    // the run-time dispatch variants exist for the float32 layout only
    // (launch_trace rejects them otherwise)
    if constexpr (kLayout == RT_LAYOUT_F32) {
        if (q.runtime_dispatch) return dispatch_runtime<kSlots, kBlock, kChunk, kQueue>(q, a, err);
    }
    switch (q.kind) {
    case RT_ISECT_DEFAULT:
        return dispatch_count<default_intersector, kSlots, kBlock, kChunk, kQueue, kLayout>(
            q, a, default_intersector::params{}, err);
    case RT_ISECT_ALPHA: {
        alpha_intersector::params p;
        p.texcoords = reinterpret_cast<const float2 *>(q.alpha.texcoords);
        p.textures = q.alpha.textures;
        p.width = q.alpha.width;
        p.height = q.alpha.height;
        p.alpha_min = q.alpha.alpha_min;
        return dispatch_count<alpha_intersector, kSlots, kBlock, kChunk, kQueue, kLayout>(q, a, p, err);
    }
    case RT_ISECT_PROCEDURAL: {
        checker_intersector::params p;
        p.n = q.checker.checker_n;
        return dispatch_count<checker_intersector, kSlots, kBlock, kChunk, kQueue, kLayout>(q, a, p,
                                                                                          err);
    }
    }
    *err = "unknown intersector kind";
    return RT_ERR_UNSUPPORTED;
}

}  // namespace

namespace {

template <class Isect, class Result>
rt_status launch_inst(const InstancedRequest &q, const kernel_args &a,
                      const typename Isect::params &p, const char **err)
{
    const uint32_t grid = (q.n_rays + 63) / 64;
    hipLaunchKernelGGL((trace_instanced_kernel<Isect, Result, kInstancedSlots>), dim3(grid), dim3(64),
                       0, static_cast<hipStream_t>(q.stream), a,
                       static_cast<const unsigned char *>(q.table), q.inst_ids, p);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        *err = hipGetErrorString(e);
        return RT_ERR_HIP;
    }
    return RT_OK;
}

template <class Isect>
rt_status launch_inst_query(const InstancedRequest &q, const kernel_args &a,
                            const typename Isect::params &p, const char **err)
{
    if (q.any) return launch_inst<Isect, any_result>(q, a, p, err);
    return launch_inst<Isect, closest_result>(q, a, p, err);
}

template <class Base>
rt_status launch_inst_count(const InstancedRequest &q, const kernel_args &a,
                            const typename Base::params &p, const char **err)
{
    if (q.count) return launch_inst_query<counting_intersector<Base>>(q, a, p, err);
    return launch_inst_query<Base>(q, a, p, err);
}

}  // namespace

rt_status launch_instanced(const InstancedRequest &q, const char **err)
{
    kernel_args a{};
    const rt_bvh_info &info = q.tlas->info;
    a.sc.nodes = static_cast<const float4 *>(q.tlas->nodes);
    a.sc.tris = static_cast<const float4 *>(q.tlas->tris);
    for (int k = 0; k < 3; ++k) {
        a.sc.root_lo[k] = info.root_lo[k];
        a.sc.root_hi[k] = info.root_hi[k];
    }
    a.sc.root_ref = info.root_ref;
    a.sc.n_tris = info.n_tris;
    a.sc.layout = info.layout;
    a.rays = static_cast<const float4 *>(q.rays);
    a.n_rays = q.n_rays;
    a.out = q.out;
    a.multi_k = 1;
    a.counters = static_cast<uint4 *>(q.counters);
    a.spill = static_cast<uint64_t *>(q.spill);
    if (q.tile_w8) {  // whole rows of 8 x 8 tiles: one wave per tile
        const uint64_t per_row = 64ull * q.tile_w8;
        a.tile_w8 = q.tile_w8;
        a.tiled = uint32_t(uint64_t(q.n_rays) / per_row * per_row);
    }
    switch (q.kind) {
    case RT_ISECT_DEFAULT:
        return launch_inst_count<default_intersector>(q, a, default_intersector::params{}, err);
    case RT_ISECT_PROCEDURAL:
        return launch_inst_count<checker_intersector>(q, a, checker_intersector::params{q.checker.checker_n},
                                                      err);
    case RT_ISECT_ALPHA: {
        alpha_intersector::params p;
        p.texcoords = nullptr;  // set per bottom-level scene at instance entry
        p.textures = q.alpha.textures;
        p.width = q.alpha.width;
        p.height = q.alpha.height;
        p.alpha_min = q.alpha.alpha_min;
        return launch_inst_count<alpha_intersector>(q, a, p, err);
    }
    default:
        break;
    }
    *err = "unknown intersector kind";
    return RT_ERR_UNSUPPORTED;
}

rt_status launch_trace(const TraceRequest &q, const char **err)
{
    kernel_args a = scene_args(*q.scene, q.rays, q.n_rays, q.out, q.counters, nullptr, q.shape);
    a.n_hits = static_cast<uint32_t *>(q.n_hits);
    a.multi_k = q.multi_k;
    a.batch = static_cast<const unsigned char *>(q.batch);
    a.spill = static_cast<uint64_t *>(q.spill);
    a.queue = static_cast<uint32_t *>(q.queue);
    if (q.tile_w8) {  // whole rows of 8 x 8 tiles of an image 8 tile_w8 wide
        const uint64_t per_row = 64ull * q.tile_w8;
        a.tile_w8 = q.tile_w8;
        a.tiled = uint32_t(uint64_t(q.n_rays) / per_row * per_row);
    }
    if (q.order) {  // longest-path-first: key and tally the chunks, then order them
        static_assert(kOrderAreaBuckets == kOrderBuckets && kOrderAreaRowChunks == kOrderRowChunks,
                      "the chunk-order area's sizing and its kernels agree");
        const uint32_t chunk = q.shape.chunk;
        const uint32_t n_chunks = uint32_t((uint64_t(q.n_rays) + chunk - 1) / chunk);
        const uint32_t n_rows = (n_chunks + kOrderRowChunks - 1) / kOrderRowChunks;
        uint32_t *keys = static_cast<uint32_t *>(q.order);
        uint32_t *order = keys + n_chunks;
        uint32_t *tallies = order + n_chunks;
        const rt_bvh_info &in = q.scene->info;
        const float dx = in.root_hi[0] - in.root_lo[0], dy = in.root_hi[1] - in.root_lo[1],
                    dz = in.root_hi[2] - in.root_lo[2];
        const float diag = std::sqrt(dx * dx + dy * dy + dz * dz);
        const float per_length = diag > 0.0f && std::isfinite(diag) ? float(kOrderBuckets) / diag : 0.0f;
        hipStream_t st = static_cast<hipStream_t>(q.stream);
        hipLaunchKernelGGL(order_keys_kernel, dim3(n_rows), dim3(kOrderKeysBlock), 0, st, a, chunk,
                           n_chunks, per_length, keys, tallies);
        hipLaunchKernelGGL(order_scatter_kernel, dim3(n_rows), dim3(kOrderScatterBlock), 0, st,
                           n_chunks, n_rows, keys, tallies, order, a.queue);
        a.order = order;
    }

    const LaunchShape &sh = q.shape;
    // 48-byte nodes: the default launch shape and its variant without the
    // queue (a lane per ray, the multi-hit query's fastest)
    if (q.scene->info.layout == RT_LAYOUT_F32P) {
        if (q.runtime_dispatch) {
            *err = "the packed node layout is compiled for the compile-time intersectors only";
            return RT_ERR_UNSUPPORTED;
        }
        if (sh.block == 64 && sh.lds_stack == 8 && sh.chunk == 64 && sh.queue == 1)
            return dispatch_kind<8, 64, 64, true, RT_LAYOUT_F32P>(q, a, err);
        if (sh.block == 64 && sh.lds_stack == 8 && sh.chunk == 64 && sh.queue == 0)
            return dispatch_kind<8, 64, 64, false, RT_LAYOUT_F32P>(q, a, err);
        *err = "the packed node layout is compiled for launch shapes (64, 8, 64, 1) and "
               "(64, 8, 64, 0) only";
        return RT_ERR_UNSUPPORTED;
    }
    // 32-byte nodes: compiled for the default launch shape only
    if (q.scene->info.layout == RT_LAYOUT_Q8) {
        constexpr LaunchShape d = kDefaultShape;
        if (sh.block != d.block || sh.lds_stack != d.lds_stack || sh.chunk != d.chunk ||
            sh.queue != d.queue || q.runtime_dispatch) {
            *err = "the compressed node layout is compiled for the default launch shape and the "
                   "compile-time intersectors only";
            return RT_ERR_UNSUPPORTED;
        }
        return dispatch_kind<int(d.lds_stack), int(d.block), int(d.chunk), d.queue != 0,
                             RT_LAYOUT_Q8>(q, a, err);
    }
    // four-wide nodes: the default launch shape and its 16-slot variant (a
    // wide node pushes up to three entries)
    if (q.scene->info.layout == RT_LAYOUT_WIDE4) {
        if (q.runtime_dispatch) {
            *err = "the four-wide node layout is compiled for the compile-time intersectors only";
            return RT_ERR_UNSUPPORTED;
        }
        if (sh.block == 64 && sh.lds_stack == 8 && sh.chunk == 64 && sh.queue == 1)
            return dispatch_kind<8, 64, 64, true, RT_LAYOUT_WIDE4>(q, a, err);
        if (sh.block == 64 && sh.lds_stack == 16 && sh.chunk == 64 && sh.queue == 1)
            return dispatch_kind<16, 64, 64, true, RT_LAYOUT_WIDE4>(q, a, err);
        *err = "the four-wide node layout is compiled for launch shapes (64, 8, 64, 1) and "
               "(64, 16, 64, 1) only";
        return RT_ERR_UNSUPPORTED;
    }
#define RTX_SHAPE(B, L, C, Q)                                                          \
    if (sh.block == B && sh.lds_stack == L && sh.chunk == C && sh.queue == Q)          \
        return dispatch_kind<L, B, C, Q>(q, a, err);
    RTX_SHAPE(64, 8, 64, 1)
    RTX_SHAPE(64, 8, 64, 0)
    RTX_SHAPE(64, 16, 64, 1)
    RTX_SHAPE(256, 8, 64, 1)
    RTX_SHAPE(128, 8, 64, 1)
    RTX_SHAPE(64, 8, 128, 1)
    RTX_SHAPE(256, 16, 64, 1)
    RTX_SHAPE(64, 8, 32, 1)
#undef RTX_SHAPE
    *err = "launch shape not compiled into the library";
    return RT_ERR_UNSUPPORTED;
}

}  // namespace rtx
