// Host-side launching of the traversal kernel template, shared by librtx and
// by C++/HIP code that compiles its own intersector into the traversal
// (Section 3.2: the intersector is a compile-time parameter of the traversal,
// so user code that includes this header gets its accept decision inlined
// into its own kernel instantiation).
//
// A user intersector derives from intersector_base and provides
//   struct params { ... };                       (passed by value to the kernel)
//   __device__ explicit T(const params &);
//   static constexpr bool kFilters = true;       (when it can reject hits)
//   __device__ bool accept(const hit_candidate &);
// and may be wrapped in counting_intersector<T> for the per-ray counters.
// trace_custom<T>() then runs the closest-hit query with it, using the
// library's default launch shape and the scene's node layout (rt_bvh_build,
// rt_bvh_compress or rt_bvh_widen).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>

#include "rt_internal.hpp"
#include "rt_traverse.hpp"

namespace rtx {

// Resident blocks per CU x CUs of the current device for `kernel` launched
// with `block` threads, cached per device in `cache`.  Each kernel
// instantiation passes its own cache: instantiations share a function-pointer
// type whenever their intersectors share a parameter type, yet differ in
// registers and block size, hence in occupancy.
template <class Kernel>
uint32_t resident_blocks(Kernel kernel, uint32_t block, std::atomic<uint32_t> (&cache)[64],
                         const char **err)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        *err = "hipGetDevice failed";
        return 0;
    }
    if (cache[dev].load(std::memory_order_relaxed) == 0) {
        int cus = 0, per_cu = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, int(block), 0) != hipSuccess ||
            cus <= 0 || per_cu <= 0) {
            *err = "occupancy query failed";
            return 0;
        }
        cache[dev].store(uint32_t(cus) * uint32_t(per_cu), std::memory_order_relaxed);
    }
    return cache[dev].load(std::memory_order_relaxed);
}

// Compute units of the current device (cached per device), or 0 with *err set.
inline uint32_t device_cus(const char **err)
{
    static std::atomic<uint32_t> cache[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        *err = "hipGetDevice failed";
        return 0;
    }
    if (cache[dev].load(std::memory_order_relaxed) == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0) {
            *err = "device attribute query failed";
            return 0;
        }
        cache[dev].store(uint32_t(cus), std::memory_order_relaxed);
    }
    return cache[dev].load(std::memory_order_relaxed);
}

// Kernel arguments for one scene; the workspace holds the queue heads (queue
// shapes) and then the stack spill columns.
inline kernel_args scene_args(const rt_scene &scene, const void *rays, uint32_t n_rays, void *out,
                              void *counters, void *workspace, const LaunchShape &shape)
{
    kernel_args a{};
    const rt_bvh_info &info = scene.info;
    a.sc.nodes = static_cast<const float4 *>(scene.nodes);
    a.sc.tris = static_cast<const float4 *>(scene.tris);
    for (int k = 0; k < 3; ++k) {
        a.sc.root_lo[k] = info.root_lo[k];
        a.sc.root_hi[k] = info.root_hi[k];
    }
    a.sc.root_ref = info.root_ref;
    a.sc.n_tris = info.n_tris;
    a.sc.layout = info.layout;
    a.rays = static_cast<const float4 *>(rays);
    a.n_rays = n_rays;
    a.out = out;
    a.multi_k = 1;
    a.counters = static_cast<uint4 *>(counters);
    unsigned char *ws = static_cast<unsigned char *>(workspace);
    a.queue = shape.queue ? reinterpret_cast<uint32_t *>(ws) : nullptr;
    a.spill = reinterpret_cast<uint64_t *>(shape.queue && ws ? ws + kQueueBytes : ws);
    return a;
}

// Enqueues one traversal kernel (and, for a queue shape, the reset of the
// queue heads before it); returns RT_OK or RT_ERR_HIP.  A queue shape's grid
// holds at most waves_per_simd waves per SIMD (4 SIMDs per CU).
template <class Isect, class Result, int kSlots, int kBlock, int kChunk, bool kQueue,
          bool kBatched = false, uint32_t kLayout = RT_LAYOUT_F32>
rt_status launch_one(const kernel_args &a, const typename Isect::params &p, hipStream_t s,
                     const char **err, uint32_t waves_per_simd = RT_DEFAULT_WAVES_PER_SIMD)
{
    const LaunchShape sh{kBlock, kSlots, kChunk, kQueue};
    auto kernel = trace_kernel<Isect, Result, kSlots, kBlock, kChunk, kQueue, kBatched, kLayout>;
    // the workspace is sized for launch_threads(); a queue grid is further
    // trimmed to the waves that can be resident at once
    uint32_t grid = uint32_t(launch_threads(a.n_rays, sh) / kBlock);
    if constexpr (kQueue) {
        static std::atomic<uint32_t> occupancy_cache[64] = {};  // this instantiation's
        const uint32_t resident = resident_blocks(kernel, kBlock, occupancy_cache, err);
        if (resident == 0) return RT_ERR_HIP;
        grid = grid < resident ? grid : resident;
        const uint32_t cus = device_cus(err);
        if (cus == 0) return RT_ERR_HIP;
        const uint32_t per_cu = 4 * waves_per_simd / uint32_t(kBlock / 64);
        const uint32_t cap = cus * (per_cu > 0 ? per_cu : 1u);
        grid = grid < cap ? grid : cap;
        // A wave draws from the queue only after its static first chunk, and
        // a drawn chunk is first_dynamic (= the grid's waves) + head + 8 k.
        // When the grid has a wave for every chunk, no draw can name a chunk,
        // whatever the heads hold, so the heads need no reset (one launch
        // less for small ray counts).  A longest-path-first order's scatter
        // kernel has zeroed them already.
        const uint64_t n_chunks = (uint64_t(a.n_rays) + kChunk - 1) / kChunk;
        if (uint64_t(grid) * (kBlock / 64) < n_chunks && a.order == nullptr)
            hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, s, a.queue);
    }
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), 0, s, a, p);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        *err = hipGetErrorString(e);
        return RT_ERR_HIP;
    }
    return RT_OK;
}

// Closest-hit query with a user intersector Isect (wrap it in
// counting_intersector<> and pass counters for the per-ray counts); with
// Result = any_result (trace_custom_any) the any-hit query.
//   scene      built by rt_bvh_build, device buffers (not validated here
//              beyond null pointers, alignment and the stack bound)
//   rays, out  device, n_rays rt_ray / rt_hit (any-hit: uint32), 16-byte
//              aligned
//   counters   device rt_counters[n_rays] iff Isect counts, else NULL
//   workspace  device, at least custom_workspace_bytes(scene, n_rays) bytes
// Returns RT_OK, RT_ERR_INVALID_ARG / RT_ERR_MISALIGNED / RT_ERR_WORKSPACE
// (nothing launched; *err says why) or RT_ERR_HIP.
inline size_t custom_workspace_bytes(const rt_scene &scene, uint32_t n_rays)
{
    return workspace_for(scene.info, n_rays, kDefaultShape);
}

template <class Isect, class Result = closest_result>
rt_status trace_custom(const rt_scene *scene, const rt_ray *rays, uint32_t n_rays,
                       const typename Isect::params &p, void *out, rt_counters *counters,
                       void *workspace, size_t workspace_bytes, hipStream_t stream,
                       const char **err)
{
    // the multi-hit policy needs the per-ray hit counts and k, which this
    // entry point does not take
    static_assert(std::is_same_v<Result, closest_result> || std::is_same_v<Result, any_result>,
                  "trace_custom runs the closest-hit or the any-hit query");
    auto is16 = [](const void *q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
    if (!scene) {
        *err = "scene is NULL";
        return RT_ERR_INVALID_ARG;
    }
    if (n_rays == 0) return RT_OK;
    if (n_rays > RT_MAX_RAYS || !rays || !out || (Isect::kCounts != (counters != nullptr))) {
        *err = "rays/out NULL, too many rays, or counters given iff the intersector counts";
        return RT_ERR_INVALID_ARG;
    }
    if (scene->info.n_tris > 0 && (!scene->tris || scene->info.max_depth >= 128)) {
        *err = "scene triangle records NULL or stack bound exceeded";
        return RT_ERR_INVALID_ARG;
    }
    if (scene->info.layout != RT_LAYOUT_F32 && scene->info.layout != RT_LAYOUT_Q8 &&
        scene->info.layout != RT_LAYOUT_WIDE4 && scene->info.layout != RT_LAYOUT_F32P) {
        *err = "unknown scene node layout";
        return RT_ERR_INVALID_ARG;
    }
    if (!is16(rays) || !is16(out) || (counters && !is16(counters)) || !is16(workspace)) {
        *err = "rays, out, counters and workspace must be 16-byte aligned";
        return RT_ERR_MISALIGNED;
    }
    if (!workspace || workspace_bytes < custom_workspace_bytes(*scene, n_rays)) {
        *err = "workspace smaller than custom_workspace_bytes";
        return RT_ERR_WORKSPACE;
    }
    constexpr LaunchShape s = kDefaultShape;
    const kernel_args a = scene_args(*scene, rays, n_rays, out, counters, workspace, s);
    if (scene->info.layout == RT_LAYOUT_Q8)
        return launch_one<Isect, Result, int(s.lds_stack), int(s.block), int(s.chunk),
                          s.queue != 0, false, RT_LAYOUT_Q8>(a, p, stream, err);
    if (scene->info.layout == RT_LAYOUT_WIDE4)
        return launch_one<Isect, Result, int(s.lds_stack), int(s.block), int(s.chunk),
                          s.queue != 0, false, RT_LAYOUT_WIDE4>(a, p, stream, err);
    if (scene->info.layout == RT_LAYOUT_F32P)
        return launch_one<Isect, Result, int(s.lds_stack), int(s.block), int(s.chunk),
                          s.queue != 0, false, RT_LAYOUT_F32P>(a, p, stream, err);
    return launch_one<Isect, Result, int(s.lds_stack), int(s.block), int(s.chunk), s.queue != 0>(
        a, p, stream, err);
}

// Any-hit query with a user intersector: occluders[i] = the first accepted
// hit's triangle (input index) or RT_MISS (uint32, device, 4-byte aligned).
template <class Isect>
rt_status trace_custom_any(const rt_scene *scene, const rt_ray *rays, uint32_t n_rays,
                           const typename Isect::params &p, uint32_t *occluders,
                           rt_counters *counters, void *workspace, size_t workspace_bytes,
                           hipStream_t stream, const char **err)
{
    return trace_custom<Isect, any_result>(scene, rays, n_rays, p, occluders, counters, workspace,
                                           workspace_bytes, stream, err);
}

}  // namespace rtx
