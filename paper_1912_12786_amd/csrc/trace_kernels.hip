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

#include "rt_internal.hpp"
#include "rt_traverse.hpp"

namespace rtx {

const LaunchShape kShapes[] = {{64, 8}, {64, 16}, {256, 8}, {256, 16}};
const uint32_t kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

struct kernel_args {
    scene_view sc;
    const float4 *rays;  // 2 float4 per ray
    uint32_t n_rays;
    void *out;           // float4 hits (closest) or uint32 occluders (any)
    uint4 *counters;
    uint2 *spill;
    uint32_t spill_stride;
};

template <class Isect, bool kAny, int kLds, int kBlock>
__global__ __launch_bounds__(kBlock) void trace_kernel(kernel_args a, typename Isect::params p)
{
    __shared__ uint2 lds[kLds][kBlock];
    const uint32_t lane = threadIdx.x;
    const uint32_t i = blockIdx.x * kBlock + lane;
    if (i >= a.n_rays) return;

    const float4 r0 = a.rays[2 * size_t(i)];
    const float4 r1 = a.rays[2 * size_t(i) + 1];
    const ray_state r = make_ray(r0, r1);
    Isect isect(p);
    trav_stack<kLds, kBlock> st{lds, a.spill, lane, i, a.spill_stride};
    const trace_result res = traverse<kAny>(a.sc, r, isect, st);

    if constexpr (kAny) {
        static_cast<uint32_t *>(a.out)[i] = res.prim;
    } else {
        static_cast<float4 *>(a.out)[i] = make_float4(res.t, __uint_as_float(res.prim), res.u, res.v);
    }
    if constexpr (Isect::kCounts)
        a.counters[i] = make_uint4(isect.num_boxes, isect.num_tris, isect.num_candidates,
                                   isect.num_accepted);
}

namespace {

template <class Isect, bool kAny, int kLds, int kBlock>
rt_status launch_one(const kernel_args &a, const typename Isect::params &p, hipStream_t s,
                     const char **err)
{
    const uint32_t grid = (a.n_rays + kBlock - 1) / kBlock;
    hipLaunchKernelGGL((trace_kernel<Isect, kAny, kLds, kBlock>), dim3(grid), dim3(kBlock), 0, s,
                       a, p);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        *err = hipGetErrorString(e);
        return RT_ERR_HIP;
    }
    return RT_OK;
}

template <class Isect, int kLds, int kBlock>
rt_status dispatch_query(const TraceRequest &q, const kernel_args &a,
                         const typename Isect::params &p, const char **err)
{
    hipStream_t s = static_cast<hipStream_t>(q.stream);
    if (q.query == Query::Any) return launch_one<Isect, true, kLds, kBlock>(a, p, s, err);
    return launch_one<Isect, false, kLds, kBlock>(a, p, s, err);
}

template <class Base, int kLds, int kBlock>
rt_status dispatch_count(const TraceRequest &q, const kernel_args &a,
                         const typename Base::params &p, const char **err)
{
    if (q.count) return dispatch_query<counting_intersector<Base>, kLds, kBlock>(q, a, p, err);
    return dispatch_query<Base, kLds, kBlock>(q, a, p, err);
}

template <int kLds, int kBlock>
rt_status dispatch_kind(const TraceRequest &q, const kernel_args &a, const char **err)
{
    switch (q.kind) {
    case RT_ISECT_DEFAULT:
        return dispatch_count<default_intersector, kLds, kBlock>(q, a, default_intersector::params{},
                                                                 err);
    case RT_ISECT_ALPHA: {
        alpha_intersector::params p;
        p.texcoords = reinterpret_cast<const float2 *>(q.alpha.texcoords);
        p.textures = q.alpha.textures;
        p.width = q.alpha.width;
        p.height = q.alpha.height;
        p.alpha_min = q.alpha.alpha_min;
        return dispatch_count<alpha_intersector, kLds, kBlock>(q, a, p, err);
    }
    case RT_ISECT_PROCEDURAL: {
        checker_intersector::params p;
        p.n = q.checker.checker_n;
        return dispatch_count<checker_intersector, kLds, kBlock>(q, a, p, err);
    }
    }
    *err = "unknown intersector kind";
    return RT_ERR_UNSUPPORTED;
}

}  // namespace

rt_status launch_trace(const TraceRequest &q, const char **err)
{
    kernel_args a;
    const rt_bvh_info &info = q.scene->info;
    a.sc.nodes = static_cast<const float4 *>(q.scene->nodes);
    a.sc.tris = static_cast<const float4 *>(q.scene->tris);
    for (int k = 0; k < 3; ++k) {
        a.sc.root_lo[k] = info.root_lo[k];
        a.sc.root_hi[k] = info.root_hi[k];
    }
    a.sc.root_ref = info.root_ref;
    a.sc.n_tris = info.n_tris;
    a.rays = static_cast<const float4 *>(q.rays);
    a.n_rays = q.n_rays;
    a.out = q.out;
    a.counters = static_cast<uint4 *>(q.counters);
    a.spill = static_cast<uint2 *>(q.spill);
    a.spill_stride = (q.n_rays + q.shape.block - 1) / q.shape.block * q.shape.block;

    const uint32_t b = q.shape.block, l = q.shape.lds_stack;
    if (b == 64 && l == 8) return dispatch_kind<8, 64>(q, a, err);
    if (b == 64 && l == 16) return dispatch_kind<16, 64>(q, a, err);
    if (b == 256 && l == 8) return dispatch_kind<8, 256>(q, a, err);
    if (b == 256 && l == 16) return dispatch_kind<16, 256>(q, a, err);
    *err = "launch shape not compiled into the library";
    return RT_ERR_UNSUPPORTED;
}

}  // namespace rtx
