// C ABI of librtx: argument validation, workspace sizing and the single
// host-side selection of the kernel instantiation per call.
#include <atomic>
#include <cmath>
#include <mutex>
#include <vector>
#include <cstdint>
#include <cstring>
#include <string>

#include <hip/hip_runtime.h>

#include "rt_internal.hpp"
#include "rt_batch_layout.hpp"

using namespace rtx;

// Fixed device scratch of rt_trace_closest_noalloc: one copy per GPU, at
// each GPU's own address.  In host code this name is only a handle for
// hipGetSymbolAddress, never a device pointer.
static __device__ __align__(256) unsigned char scratch[RT_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_last_error;

// Flag bits every single-scene trace call knows: the intersector options and
// the launch-shape field.
constexpr uint32_t kKnownFlags = RT_FLAG_COUNT | RT_FLAG_RUNTIME_SWITCH | RT_FLAG_RUNTIME_CALL |
                                 RT_FLAG_SHAPE_MASK | RT_FLAG_TILE_MASK | RT_FLAG_LONGEST_FIRST |
                                 RT_FLAG_WAVES_MASK;

rt_status fail(rt_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

// The launch shape a call's flags select (RT_FLAG_SHAPE); false if the index
// names no compiled shape.
bool shape_of(uint32_t flags, LaunchShape &out)
{
    const uint32_t i = (flags & RT_FLAG_SHAPE_MASK) >> RT_FLAG_SHAPE_SHIFT;
    if (i >= kNumShapes) return false;
    out = kShapes[i];
    return true;
}

bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

rt_status check_scene(const rt_scene *sc)
{
    if (!sc) return fail(RT_ERR_INVALID_ARG, "scene is NULL");
    const rt_bvh_info &in = sc->info;
    if (in.n_tris > RT_MAX_TRIS) return fail(RT_ERR_INVALID_ARG, "scene has more than 2^29-1 triangles");
    if (in.n_tris == 0) return RT_OK;
    if (!sc->tris) return fail(RT_ERR_INVALID_ARG, "scene triangle records are NULL");
    if (!aligned(sc->tris, 16)) return fail(RT_ERR_MISALIGNED, "scene triangle records not 16-byte aligned");
    if (in.max_depth >= 128) return fail(RT_ERR_INVALID_ARG, "scene max_depth must be < 128");
    if (in.layout != RT_LAYOUT_F32 && in.layout != RT_LAYOUT_Q8 && in.layout != RT_LAYOUT_WIDE4 &&
        in.layout != RT_LAYOUT_F32P)
        return fail(RT_ERR_INVALID_ARG, "unknown scene node layout");
    const uint32_t cnt = in.root_ref >> 29, idx = in.root_ref & 0x1FFFFFFFu;
    if (cnt == 0) {
        if (in.n_nodes == 0 || idx >= in.n_nodes)
            return fail(RT_ERR_INVALID_ARG, "scene root references a missing inner node");
        if (!sc->nodes) return fail(RT_ERR_INVALID_ARG, "scene nodes are NULL");
        if (!aligned(sc->nodes, 16)) return fail(RT_ERR_MISALIGNED, "scene nodes not 16-byte aligned");
        if (in.n_nodes >= in.n_tris) return fail(RT_ERR_INVALID_ARG, "scene has more inner nodes than triangles");
    } else {
        // rt_bvh_build_ex records its leaf limit; 0 (a hand-made info) means 4
        const uint32_t leaf_cap = in.max_leaf ? in.max_leaf : 4u;
        if (in.max_leaf > 7 || cnt > leaf_cap || uint64_t(idx) + cnt > in.n_tris)
            return fail(RT_ERR_INVALID_ARG, "scene root leaf out of range");
    }
    return RT_OK;
}

rt_status check_alpha(const rt_scene *sc, const rt_alpha_params &p)
{
    if (!p.texcoords || !p.textures) return fail(RT_ERR_INVALID_ARG, "alpha texcoords/textures are NULL");
    if (!aligned(p.texcoords, 8)) return fail(RT_ERR_MISALIGNED, "alpha texcoords not 8-byte aligned");
    if (!aligned(p.textures, 4)) return fail(RT_ERR_MISALIGNED, "alpha textures not 4-byte aligned");
    if (p.n_texcoord_prims < sc->info.n_tris)
        return fail(RT_ERR_INVALID_ARG, "alpha texcoords cover fewer triangles than the scene");
    if (sc->info.n_tris > 0 && p.n_tex <= sc->info.max_geom_id)
        return fail(RT_ERR_INVALID_ARG, "alpha n_tex must exceed the scene's max geom_id");
    if (p.width < 1 || p.height < 1 || p.width > (1u << 24) || p.height > (1u << 24))
        return fail(RT_ERR_INVALID_ARG, "alpha texture size must be within 1..2^24");
    if (p.alpha_min > 255) return fail(RT_ERR_INVALID_ARG, "alpha_min must be 0..255");
    return RT_OK;
}

rt_status check_params(const rt_scene *sc, rt_isect_kind kind, const void *params, TraceRequest &q)
{
    q.kind = kind;
    std::memset(&q.alpha, 0, sizeof q.alpha);
    q.checker.checker_n = 0;
    switch (kind) {
    case RT_ISECT_DEFAULT:
        return RT_OK;
    case RT_ISECT_ALPHA: {
        if (!params) return fail(RT_ERR_INVALID_ARG, "alpha intersector needs rt_alpha_params");
        const rt_alpha_params &p = *static_cast<const rt_alpha_params *>(params);
        const rt_status st = check_alpha(sc, p);
        if (st != RT_OK) return st;
        q.alpha = p;
        return RT_OK;
    }
    case RT_ISECT_PROCEDURAL: {
        if (!params) return fail(RT_ERR_INVALID_ARG, "procedural intersector needs rt_procedural_params");
        const rt_procedural_params &p = *static_cast<const rt_procedural_params *>(params);
        if (p.checker_n < 1 || p.checker_n > 65536)
            return fail(RT_ERR_INVALID_ARG, "checker_n must be within 1..65536");
        q.checker = p;
        return RT_OK;
    }
    }
    return fail(RT_ERR_UNSUPPORTED, "unknown intersector kind");
}

// Device address of `scratch` on each device, looked up once per device
// with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

rt_status scratch_on_current_device(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(RT_ERR_HIP, "no current HIP device for the fixed scratch");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(RT_ERR_HIP, std::string("hipGetSymbolAddress of the fixed scratch: ") +
                                        hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RT_OK;
}

rt_status trace_common(Query query, const rt_scene *scene, const rt_ray *rays, uint32_t n_rays,
                       rt_isect_kind kind, const void *params, uint32_t flags, void *out,
                       size_t out_align, rt_counters *counters, void *workspace,
                       size_t workspace_bytes, void *stream, uint32_t multi_k = 0,
                       uint32_t *n_hits = nullptr, const void *batch = nullptr,
                       bool fixed_scratch = false)
{
    g_last_error.clear();
    rt_status st = check_scene(scene);
    if (st != RT_OK) return st;
    if (flags & ~kKnownFlags) return fail(RT_ERR_UNSUPPORTED, "unknown flag bits");
    LaunchShape shape;
    if (!shape_of(flags, shape)) return fail(RT_ERR_UNSUPPORTED, "launch shape index not compiled in");
    const uint32_t runtime = flags & (RT_FLAG_RUNTIME_SWITCH | RT_FLAG_RUNTIME_CALL);
    if (runtime) {
        if (runtime == (RT_FLAG_RUNTIME_SWITCH | RT_FLAG_RUNTIME_CALL))
            return fail(RT_ERR_INVALID_ARG, "choose one runtime dispatch flag");
        if (query != Query::Closest || batch || (flags & RT_FLAG_COUNT))
            return fail(RT_ERR_UNSUPPORTED,
                        "runtime dispatch is compiled for the plain closest-hit query only");
    }
    TraceRequest q;
    q.runtime_dispatch = runtime == RT_FLAG_RUNTIME_SWITCH ? 1u : (runtime ? 2u : 0u);
    q.tile_w8 = (flags & RT_FLAG_TILE_MASK) >> RT_FLAG_TILE_SHIFT;
    const uint32_t waves = (flags & RT_FLAG_WAVES_MASK) >> RT_FLAG_WAVES_SHIFT;
    q.waves_per_simd = waves ? waves : RT_DEFAULT_WAVES_PER_SIMD;
    if (q.tile_w8 && batch)
        return fail(RT_ERR_UNSUPPORTED, "the tiled schedule is for single-scene calls");
    const bool longest_first = (flags & RT_FLAG_LONGEST_FIRST) != 0;
    if (longest_first && batch)
        return fail(RT_ERR_UNSUPPORTED, "the longest-path-first schedule is for single-scene calls");
    if (batch) {  // per-scene data was validated by rt_batch_pack
        q.kind = kind;
        std::memset(&q.alpha, 0, sizeof q.alpha);
        q.checker.checker_n =
            kind == RT_ISECT_PROCEDURAL ? static_cast<const rt_procedural_params *>(params)->checker_n : 0;
    } else {
        st = check_params(scene, kind, params, q);
        if (st != RT_OK) return st;
    }
    if (query == Query::Multi && (multi_k < 1 || multi_k > RT_MAX_MULTI))
        return fail(RT_ERR_INVALID_ARG, "multi-hit k must be within 1..RT_MAX_MULTI");
    if (n_rays == 0) return RT_OK;
    if (n_rays > RT_MAX_RAYS) return fail(RT_ERR_INVALID_ARG, "more than 2^31 rays in one call");
    if (query == Query::Multi && (!n_hits || !aligned(n_hits, 4)))
        return fail(RT_ERR_INVALID_ARG, "multi-hit needs a 4-byte aligned n_hits array");
    if (!rays) return fail(RT_ERR_INVALID_ARG, "rays are NULL");
    if (!aligned(rays, 16)) return fail(RT_ERR_MISALIGNED, "rays not 16-byte aligned");
    if (!out) return fail(RT_ERR_INVALID_ARG, "output array is NULL");
    if (!aligned(out, out_align)) return fail(RT_ERR_MISALIGNED, "output array misaligned");
    const bool count = (flags & RT_FLAG_COUNT) != 0;
    if (count && !counters) return fail(RT_ERR_INVALID_ARG, "RT_FLAG_COUNT needs a counters array");
    if (count && !aligned(counters, 16)) return fail(RT_ERR_MISALIGNED, "counters not 16-byte aligned");
    const size_t need = workspace_for(scene->info, n_rays, shape, longest_first);
    if (fixed_scratch) {  // the library's own scratch replaces the workspace
        if (need > RT_NOALLOC_SCRATCH_BYTES)
            return fail(RT_ERR_WORKSPACE,
                        "call needs " + std::to_string(need) + " bytes of workspace, more than "
                        "the fixed scratch of rt_trace_closest_noalloc (" +
                        std::to_string(RT_NOALLOC_SCRATCH_BYTES) + "): use rt_trace_closest "
                        "with a workspace, a launch shape with more LDS stack slots, or fewer "
                        "rays per call");
        workspace = nullptr;
        workspace_bytes = 0;
        if (need > 0) {
            st = scratch_on_current_device(&workspace);
            if (st != RT_OK) return st;
            workspace_bytes = RT_NOALLOC_SCRATCH_BYTES;
        }
    } else if (need > 0) {
        if (!workspace || workspace_bytes < need)
            return fail(RT_ERR_WORKSPACE, "workspace smaller than rt_trace_workspace_bytes");
        if (!aligned(workspace, 16)) return fail(RT_ERR_MISALIGNED, "workspace not 16-byte aligned");
    }
    q.scene = scene;
    q.rays = rays;
    q.n_rays = n_rays;
    q.count = count;
    q.query = query;
    q.out = out;
    q.n_hits = n_hits;
    q.multi_k = query == Query::Multi ? multi_k : 1;
    q.counters = count ? counters : nullptr;
    q.batch = batch;
    // workspace: [queue heads][chunk-order area][spill columns]
    char *w = static_cast<char *>(workspace);
    q.queue = shape.queue ? w : nullptr;
    w += shape.queue ? kQueueBytes : 0;
    q.order = longest_first ? w : nullptr;
    w += longest_first ? order_bytes(n_rays, shape) : 0;
    q.spill = w;
    q.shape = shape;
    q.stream = stream;
    const char *err = "";
    st = launch_trace(q, &err);
    if (st != RT_OK) return fail(st, err);
    return RT_OK;
}

}  // namespace

extern "C" {

rt_status rt_bvh_buffer_bytes(uint32_t n_tris, size_t *node_bytes, size_t *tri_bytes)
{
    g_last_error.clear();
    if (!node_bytes || !tri_bytes) return fail(RT_ERR_INVALID_ARG, "output pointers are NULL");
    if (n_tris > RT_MAX_TRIS) return fail(RT_ERR_INVALID_ARG, "more than 2^29-1 triangles");
    *node_bytes = size_t(max_inner_nodes(n_tris, 1)) * RT_NODE_BYTES;
    *tri_bytes = size_t(n_tris) * RT_TRI_BYTES;
    return RT_OK;
}

rt_status rt_bvh_build(const float *vertices, const uint32_t *geom_ids, uint32_t n_tris,
                       void *nodes, size_t node_cap, void *tris, size_t tri_cap, rt_bvh_info *info)
{
    return rt_bvh_build_ex(vertices, geom_ids, n_tris, nullptr, nodes, node_cap, tris, tri_cap, info);
}

rt_status rt_bvh_build_ex(const float *vertices, const uint32_t *geom_ids, uint32_t n_tris,
                          const rt_build_params *params, void *nodes, size_t node_cap, void *tris,
                          size_t tri_cap, rt_bvh_info *info)
{
    g_last_error.clear();
    if (!info) return fail(RT_ERR_INVALID_ARG, "info is NULL");
    const uint32_t max_leaf = params ? params->max_leaf : 4u;
    if (max_leaf < 1 || max_leaf > 7) return fail(RT_ERR_INVALID_ARG, "max_leaf must be within 1..7");
    if (n_tris > RT_MAX_TRIS) return fail(RT_ERR_INVALID_ARG, "more than 2^29-1 triangles");
    if (n_tris > 0 && !vertices) return fail(RT_ERR_INVALID_ARG, "vertices are NULL");
    const size_t need_nodes = size_t(max_inner_nodes(n_tris, max_leaf)) * RT_NODE_BYTES;
    const size_t need_tris = size_t(n_tris) * RT_TRI_BYTES;
    if (need_nodes > 0 && (!nodes || node_cap < need_nodes))
        return fail(RT_ERR_INVALID_ARG, "node buffer smaller than rt_bvh_buffer_bytes");
    if (need_tris > 0 && (!tris || tri_cap < need_tris))
        return fail(RT_ERR_INVALID_ARG, "triangle buffer smaller than rt_bvh_buffer_bytes");
    if ((nodes && !aligned(nodes, 16)) || (tris && !aligned(tris, 16)))
        return fail(RT_ERR_MISALIGNED, "host output buffers must be 16-byte aligned");
    rt_status st = build_bvh(vertices, geom_ids, n_tris, max_leaf, static_cast<NodeRecord *>(nodes),
                             static_cast<TriRecord *>(tris), info);
    if (st != RT_OK) return fail(st, "host allocation failed during BVH build");
    return RT_OK;
}

rt_status rt_bvh_compress(const void *nodes, const rt_bvh_info *info, void *out, size_t out_cap,
                          rt_bvh_info *out_info)
{
    g_last_error.clear();
    if (!info || !out_info) return fail(RT_ERR_INVALID_ARG, "info/out_info are NULL");
    if (info->layout != RT_LAYOUT_F32) return fail(RT_ERR_INVALID_ARG, "input nodes are not RT_LAYOUT_F32");
    const size_t need = size_t(info->n_nodes) * RT_NODE_BYTES_Q8;
    if (info->n_nodes > 0) {
        if (!nodes || !out) return fail(RT_ERR_INVALID_ARG, "nodes/out are NULL");
        if (out_cap < need) return fail(RT_ERR_INVALID_ARG, "out smaller than n_nodes * RT_NODE_BYTES_Q8");
        if (!aligned(nodes, 16) || !aligned(out, 16))
            return fail(RT_ERR_MISALIGNED, "nodes/out must be 16-byte aligned");
        const rt_status st = compress_nodes(static_cast<const NodeRecord *>(nodes), info->n_nodes,
                                            static_cast<NodeQ8Record *>(out));
        if (st != RT_OK) return fail(st, "a node box is not finite");
    }
    rt_bvh_info o = *info;
    o.layout = RT_LAYOUT_Q8;
    *out_info = o;
    return RT_OK;
}

rt_status rt_bvh_refit_plan(const void *nodes, const rt_bvh_info *info, uint32_t *plan,
                            size_t plan_cap, uint32_t *n_top)
{
    g_last_error.clear();
    if (!info || !n_top) return fail(RT_ERR_INVALID_ARG, "info/n_top are NULL");
    if (info->layout != RT_LAYOUT_F32) return fail(RT_ERR_UNSUPPORTED, "refit takes RT_LAYOUT_F32 trees");
    *n_top = 0;
    if (info->n_nodes == 0 || (info->root_ref >> 29) != 0) return RT_OK;  // a root leaf
    if (!nodes || !plan) return fail(RT_ERR_INVALID_ARG, "nodes/plan are NULL");
    if (plan_cap < 3 * size_t(info->n_nodes))
        return fail(RT_ERR_INVALID_ARG, "plan smaller than 3 * n_nodes words");
    if ((info->root_ref & kRefIndexMaskHost) != 0)
        return fail(RT_ERR_INVALID_ARG, "the root is not node 0 (not a tree from rt_bvh_build)");
    const uint32_t t = refit_plan(static_cast<const NodeRecord *>(nodes), *info, plan);
    if (t == UINT32_MAX)
        return fail(RT_ERR_INVALID_ARG, "a child reference is not a later node, or a node is not "
                                        "the child of exactly one node");
    *n_top = t;
    return RT_OK;
}

rt_status rt_bvh_refit(const rt_scene *scene, const uint32_t *plan, uint32_t n_top,
                       const float *vertices, uint32_t n_vertices, const uint32_t *faces,
                       float *root_box, void *stream)
{
    g_last_error.clear();
    rt_status st = check_scene(scene);
    if (st != RT_OK) return st;
    const rt_bvh_info &in = scene->info;
    if (in.layout != RT_LAYOUT_F32) return fail(RT_ERR_UNSUPPORTED, "refit takes RT_LAYOUT_F32 scenes");
    if (in.n_tris == 0) return RT_OK;
    if (!vertices || !faces || !root_box) return fail(RT_ERR_INVALID_ARG, "vertices/faces/root_box are NULL");
    if (!aligned(vertices, 4) || !aligned(faces, 4) || !aligned(root_box, 4))
        return fail(RT_ERR_MISALIGNED, "vertices, faces and root_box must be 4-byte aligned");
    RefitRequest q{};
    if ((in.root_ref >> 29) == 0) {
        if (!plan) return fail(RT_ERR_INVALID_ARG, "an inner root needs the plan");
        if (!aligned(plan, 4)) return fail(RT_ERR_MISALIGNED, "plan must be 4-byte aligned");
        if ((in.root_ref & kRefIndexMaskHost) != 0)
            return fail(RT_ERR_INVALID_ARG, "the root is not node 0 (not a tree from rt_bvh_build)");
        if (n_top > in.n_nodes) return fail(RT_ERR_INVALID_ARG, "n_top exceeds n_nodes");
        if (in.n_nodes > kRefitBlockNodes && n_top == 0)
            return fail(RT_ERR_INVALID_ARG, "a tree of more than one refit block has top nodes");
        q.n_nodes = in.n_nodes;
    } else {
        q.root_first = in.root_ref & kRefIndexMaskHost;
        q.root_count = in.root_ref >> 29;
    }
    q.nodes = const_cast<void *>(scene->nodes);
    q.max_depth = in.max_depth;
    q.tris = const_cast<void *>(scene->tris);
    q.n_tris = in.n_tris;
    q.plan = plan;
    q.n_top = n_top;
    q.vertices = vertices;
    q.n_vertices = n_vertices;
    q.faces = faces;
    q.root_box = root_box;
    q.stream = stream;
    const char *err = "";
    st = launch_refit(q, &err);
    if (st != RT_OK) return fail(st, err);
    return RT_OK;
}

rt_status rt_bvh_pack(const void *nodes, const rt_bvh_info *info, void *out, size_t out_cap,
                      rt_bvh_info *out_info)
{
    g_last_error.clear();
    if (!info || !out_info) return fail(RT_ERR_INVALID_ARG, "info/out_info are NULL");
    if (info->layout != RT_LAYOUT_F32) return fail(RT_ERR_INVALID_ARG, "input nodes are not RT_LAYOUT_F32");
    const size_t need = size_t(info->n_nodes) * RT_NODE_BYTES_F32P;
    if (info->n_nodes > 0) {
        if (!nodes || !out) return fail(RT_ERR_INVALID_ARG, "nodes/out are NULL");
        if (out_cap < need) return fail(RT_ERR_INVALID_ARG, "out smaller than n_nodes * RT_NODE_BYTES_F32P");
        if (!aligned(nodes, 16) || !aligned(out, 16))
            return fail(RT_ERR_MISALIGNED, "nodes/out must be 16-byte aligned");
        const rt_status st = pack_nodes(static_cast<const NodeRecord *>(nodes), info->n_nodes,
                                        static_cast<NodePackedRecord *>(out));
        if (st != RT_OK)
            return fail(st, "a node box is not finite or too close to the float range's end");
    }
    rt_bvh_info o = *info;
    o.layout = RT_LAYOUT_F32P;
    *out_info = o;
    return RT_OK;
}

rt_status rt_bvh_widen(const void *nodes, const rt_bvh_info *info, void *out, size_t out_cap,
                       rt_bvh_info *out_info)
{
    g_last_error.clear();
    if (!info || !out_info) return fail(RT_ERR_INVALID_ARG, "info/out_info are NULL");
    if (info->layout != RT_LAYOUT_F32) return fail(RT_ERR_INVALID_ARG, "input nodes are not RT_LAYOUT_F32");
    rt_bvh_info o = *info;
    o.layout = RT_LAYOUT_WIDE4;
    if ((info->root_ref >> 29) == 0 && info->n_nodes > 0) {
        const size_t need = size_t(info->n_nodes) * RT_NODE_BYTES_WIDE4;
        if (!nodes || !out) return fail(RT_ERR_INVALID_ARG, "nodes/out are NULL");
        if (out_cap < need) return fail(RT_ERR_INVALID_ARG, "out smaller than n_nodes * RT_NODE_BYTES_WIDE4");
        if (!aligned(nodes, 16) || !aligned(out, 16))
            return fail(RT_ERR_MISALIGNED, "nodes/out must be 16-byte aligned");
        uint32_t n_wide = 0, bound = 0;
        const rt_status st = widen_nodes(static_cast<const NodeRecord *>(nodes), *info,
                                         static_cast<NodeW4Record *>(out), &n_wide, &bound);
        if (st != RT_OK) return fail(st, "a child reference is out of range");
        o.n_nodes = n_wide;
        o.max_depth = bound;
        o.root_ref = 0;
    } else {
        o.n_nodes = 0;
        o.max_depth = 0;
    }
    *out_info = o;
    return RT_OK;
}

rt_status rt_trace_workspace_bytes(const rt_scene *scene, uint32_t n_rays, uint32_t flags,
                                   size_t *bytes)
{
    g_last_error.clear();
    if (!bytes) return fail(RT_ERR_INVALID_ARG, "bytes is NULL");
    rt_status st = check_scene(scene);
    if (st != RT_OK) return st;
    // the runtime-dispatch flags select kernels with the same workspace
    if (flags & ~kKnownFlags) return fail(RT_ERR_UNSUPPORTED, "unknown flag bits");
    LaunchShape shape;
    if (!shape_of(flags, shape)) return fail(RT_ERR_UNSUPPORTED, "launch shape index not compiled in");
    if (n_rays > RT_MAX_RAYS) return fail(RT_ERR_INVALID_ARG, "more than 2^31 rays in one call");
    *bytes = workspace_for(scene->info, n_rays, shape, (flags & RT_FLAG_LONGEST_FIRST) != 0);
    return RT_OK;
}

rt_status rt_trace_closest(const rt_scene *scene, const rt_ray *rays, uint32_t n_rays,
                           rt_isect_kind kind, const void *params, uint32_t flags, rt_hit *hits,
                           rt_counters *counters, void *workspace, size_t workspace_bytes,
                           void *stream)
{
    return trace_common(Query::Closest, scene, rays, n_rays, kind, params, flags, hits, 16,
                        counters, workspace, workspace_bytes, stream);
}

rt_status rt_trace_closest_noalloc(const rt_scene *scene, const rt_ray *rays, uint32_t n_rays,
                                   rt_isect_kind kind, const void *params, uint32_t flags,
                                   rt_hit *hits, rt_counters *counters, void *stream)
{
    return trace_common(Query::Closest, scene, rays, n_rays, kind, params, flags, hits, 16,
                        counters, nullptr, 0, stream, 0, nullptr, nullptr, true);
}

rt_status rt_trace_any(const rt_scene *scene, const rt_ray *rays, uint32_t n_rays,
                       rt_isect_kind kind, const void *params, uint32_t flags, uint32_t *occluder,
                       rt_counters *counters, void *workspace, size_t workspace_bytes, void *stream)
{
    return trace_common(Query::Any, scene, rays, n_rays, kind, params, flags, occluder, 4,
                        counters, workspace, workspace_bytes, stream);
}

rt_status rt_batch_table_bytes(uint32_t n_scenes, size_t *bytes)
{
    g_last_error.clear();
    if (!bytes) return fail(RT_ERR_INVALID_ARG, "bytes is NULL");
    if (n_scenes == 0 || n_scenes > (1u << 24)) return fail(RT_ERR_INVALID_ARG, "n_scenes must be 1..2^24");
    *bytes = batch_records_offset(n_scenes) + size_t(n_scenes) * sizeof(batch_scene);
    return RT_OK;
}

rt_status rt_batch_pack(const rt_batch_entry *entries, uint32_t n_scenes, rt_isect_kind kind,
                        void *host_table, size_t table_bytes, rt_batch_info *info)
{
    g_last_error.clear();
    size_t need = 0;
    rt_status st = rt_batch_table_bytes(n_scenes, &need);
    if (st != RT_OK) return st;
    if (!entries || !host_table || !info) return fail(RT_ERR_INVALID_ARG, "entries/table/info are NULL");
    if (table_bytes < need) return fail(RT_ERR_INVALID_ARG, "table smaller than rt_batch_table_bytes");
    if (!aligned(host_table, 16)) return fail(RT_ERR_MISALIGNED, "table not 16-byte aligned");
    if (kind != RT_ISECT_DEFAULT && kind != RT_ISECT_ALPHA && kind != RT_ISECT_PROCEDURAL)
        return fail(RT_ERR_UNSUPPORTED, "unknown intersector kind");
    unsigned char *t = static_cast<unsigned char *>(host_table);
    std::memset(t, 0, need);
    uint32_t *header = reinterpret_cast<uint32_t *>(t);
    uint32_t *prefix = reinterpret_cast<uint32_t *>(t + batch_prefix_offset());
    batch_scene *rec = reinterpret_cast<batch_scene *>(t + batch_records_offset(n_scenes));
    header[0] = n_scenes;
    uint64_t total = 0;
    uint32_t depth = 0;
    const uint32_t layout = n_scenes ? entries[0].scene.info.layout : RT_LAYOUT_F32;
    for (uint32_t s = 0; s < n_scenes; ++s) {
        const rt_batch_entry &e = entries[s];
        st = check_scene(&e.scene);
        if (st != RT_OK) return fail(st, "scene " + std::to_string(s) + ": " + g_last_error);
        if (e.scene.info.layout != layout)
            return fail(RT_ERR_UNSUPPORTED, "scene " + std::to_string(s) +
                                                ": the scenes of a batch must share one node layout");
        if (kind == RT_ISECT_ALPHA) {
            st = check_alpha(&e.scene, e.alpha);
            if (st != RT_OK) return fail(st, "scene " + std::to_string(s) + ": " + g_last_error);
        }
        prefix[s] = uint32_t(total);
        total += e.n_rays;
        if (total > RT_MAX_RAYS) return fail(RT_ERR_INVALID_ARG, "more than 2^31 rays in one batch");
        const rt_bvh_info &in = e.scene.info;
        batch_scene &r = rec[s];
        r.nodes = static_cast<const float4 *>(e.scene.nodes);
        r.tris = static_cast<const float4 *>(e.scene.tris);
        r.texcoords = reinterpret_cast<const float2 *>(e.alpha.texcoords);
        r.textures = e.alpha.textures;
        for (int a = 0; a < 3; ++a) {
            r.root_lo[a] = in.root_lo[a];
            r.root_hi[a] = in.root_hi[a];
        }
        r.root_ref = in.root_ref;
        r.n_tris = in.n_tris;
        r.layout = in.layout;
        r.tex_width = e.alpha.width;
        r.tex_height = e.alpha.height;
        r.alpha_min = e.alpha.alpha_min;
        depth = in.max_depth > depth ? in.max_depth : depth;
    }
    prefix[n_scenes] = uint32_t(total);
    info->n_scenes = n_scenes;
    info->n_rays = uint32_t(total);
    info->max_depth = depth;
    info->kind = uint32_t(kind);
    info->layout = layout;
    return RT_OK;
}

rt_status rt_trace_batch_workspace_bytes(const rt_batch_info *info, uint32_t flags, size_t *bytes)
{
    g_last_error.clear();
    if (!info || !bytes) return fail(RT_ERR_INVALID_ARG, "info/bytes are NULL");
    if (flags & ~(RT_FLAG_COUNT | RT_FLAG_SHAPE_MASK | RT_FLAG_WAVES_MASK))
        return fail(RT_ERR_UNSUPPORTED, "unknown flag bits");
    LaunchShape shape;
    if (!shape_of(flags, shape)) return fail(RT_ERR_UNSUPPORTED, "launch shape index not compiled in");
    rt_bvh_info bi{};
    bi.max_depth = info->max_depth;
    *bytes = workspace_for(bi, info->n_rays, shape);
    return RT_OK;
}

rt_status rt_trace_batch(const void *table, const rt_batch_info *info, const rt_ray *rays,
                         rt_isect_kind kind, const void *params, uint32_t flags, rt_hit *hits,
                         rt_counters *counters, void *workspace, size_t workspace_bytes,
                         void *stream)
{
    g_last_error.clear();
    if (!info) return fail(RT_ERR_INVALID_ARG, "info is NULL");
    if (!table) return fail(RT_ERR_INVALID_ARG, "table is NULL");
    if (!aligned(table, 16)) return fail(RT_ERR_MISALIGNED, "table not 16-byte aligned");
    if (uint32_t(kind) != info->kind)
        return fail(RT_ERR_INVALID_ARG, "kind differs from the kind the table was packed for");
    if (info->max_depth >= 128) return fail(RT_ERR_INVALID_ARG, "batch max_depth must be < 128");
    if (kind == RT_ISECT_ALPHA && params)
        return fail(RT_ERR_INVALID_ARG, "a batched alpha launch takes its data from the table");
    if (kind == RT_ISECT_PROCEDURAL) {
        if (!params) return fail(RT_ERR_INVALID_ARG, "procedural intersector needs rt_procedural_params");
        const uint32_t n = static_cast<const rt_procedural_params *>(params)->checker_n;
        if (n < 1 || n > 65536) return fail(RT_ERR_INVALID_ARG, "checker_n must be within 1..65536");
    } else if (kind != RT_ISECT_DEFAULT && kind != RT_ISECT_ALPHA) {
        return fail(RT_ERR_UNSUPPORTED, "unknown intersector kind");
    }
    // a stand-in scene carries the batch-wide sizes through the common checks
    if (info->layout != RT_LAYOUT_F32 && info->layout != RT_LAYOUT_Q8 &&
        info->layout != RT_LAYOUT_WIDE4 && info->layout != RT_LAYOUT_F32P)
        return fail(RT_ERR_INVALID_ARG, "unknown batch node layout");
    rt_scene proxy{};
    proxy.info.max_depth = info->max_depth;
    proxy.info.layout = info->layout;
    return trace_common(Query::Closest, &proxy, rays, info->n_rays, kind, params, flags, hits, 16,
                        counters, workspace, workspace_bytes, stream, 0, nullptr, table);
}

rt_status rt_tlas_build(const rt_instance *instances, uint32_t n_inst, void *nodes,
                        size_t node_cap, void *tris, size_t tri_cap, rt_bvh_info *info)
{
    g_last_error.clear();
    if (n_inst > 0 && !instances) return fail(RT_ERR_INVALID_ARG, "instances are NULL");
    if (n_inst > RT_MAX_TRIS) return fail(RT_ERR_INVALID_ARG, "more than 2^29-1 instances");
    std::vector<float> boxes;
    try {
        boxes.resize(size_t(n_inst) * 9);
    } catch (const std::bad_alloc &) {
        return fail(RT_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    for (uint32_t q = 0; q < n_inst; ++q) {
        const rt_instance &in = instances[q];
        for (int a = 0; a < 3; ++a) {
            const float lo = in.world_lo[a], hi = in.world_hi[a];
            if (!std::isfinite(lo) || !std::isfinite(hi) || lo > hi)
                return fail(RT_ERR_INVALID_ARG, "instance " + std::to_string(q) + ": bad world box");
            // the box as the degenerate triangle (lo, hi, hi)
            boxes[9 * size_t(q) + a] = lo;
            boxes[9 * size_t(q) + 3 + a] = hi;
            boxes[9 * size_t(q) + 6 + a] = hi;
        }
    }
    return rt_bvh_build(boxes.data(), nullptr, n_inst, nodes, node_cap, tris, tri_cap, info);
}

rt_status rt_instance_table_bytes(uint32_t n_blas, uint32_t n_inst, size_t *bytes)
{
    g_last_error.clear();
    if (!bytes) return fail(RT_ERR_INVALID_ARG, "bytes is NULL");
    if (n_blas > (1u << 24) || n_inst > RT_MAX_TRIS)
        return fail(RT_ERR_INVALID_ARG, "too many bottom-level scenes or instances");
    *bytes = instance_records_offset(n_blas) + size_t(n_inst) * sizeof(instance_record);
    return RT_OK;
}

rt_status rt_instance_pack(const rt_scene *blas, const rt_mesh_texcoords *texcoords,
                           uint32_t n_blas, const rt_instance *instances, uint32_t n_inst,
                           void *host_table, size_t table_bytes, rt_instance_info *info)
{
    size_t need = 0;
    rt_status st = rt_instance_table_bytes(n_blas, n_inst, &need);
    if (st != RT_OK) return st;
    if ((n_blas && !blas) || (n_inst && !instances) || !host_table || !info)
        return fail(RT_ERR_INVALID_ARG, "blas/instances/table/info are NULL");
    if (table_bytes < need) return fail(RT_ERR_INVALID_ARG, "table smaller than rt_instance_table_bytes");
    if (!aligned(host_table, 16)) return fail(RT_ERR_MISALIGNED, "table not 16-byte aligned");
    unsigned char *t = static_cast<unsigned char *>(host_table);
    std::memset(t, 0, need);
    uint32_t *hdr = reinterpret_cast<uint32_t *>(t);
    hdr[0] = n_blas;
    hdr[1] = n_inst;
    blas_record *br = reinterpret_cast<blas_record *>(t + instance_blas_offset());
    instance_record *ir = reinterpret_cast<instance_record *>(t + instance_records_offset(n_blas));
    rt_instance_info out{};
    out.n_blas = n_blas;
    out.n_inst = n_inst;
    out.has_texcoords = texcoords ? 1u : 0u;
    for (uint32_t b = 0; b < n_blas; ++b) {
        const std::string which = "bottom-level scene " + std::to_string(b);
        st = check_scene(&blas[b]);
        if (st != RT_OK) return fail(st, which + ": " + g_last_error);
        if (blas[b].info.layout != RT_LAYOUT_F32)
            return fail(RT_ERR_UNSUPPORTED, which + ": instancing takes RT_LAYOUT_F32 scenes");
        const rt_bvh_info &in = blas[b].info;
        br[b].nodes = static_cast<const float4 *>(blas[b].nodes);
        br[b].tris = static_cast<const float4 *>(blas[b].tris);
        for (int a = 0; a < 3; ++a) {
            br[b].root_lo[a] = in.root_lo[a];
            br[b].root_hi[a] = in.root_hi[a];
        }
        br[b].root_ref = in.root_ref;
        br[b].n_tris = in.n_tris;
        br[b].layout = in.layout;
        if (texcoords && in.n_tris > 0) {
            const rt_mesh_texcoords &tc = texcoords[b];
            if (!tc.texcoords || tc.n_prims < in.n_tris)
                return fail(RT_ERR_INVALID_ARG, which + ": texcoords NULL or covering fewer triangles");
            if (!aligned(tc.texcoords, 8))
                return fail(RT_ERR_MISALIGNED, which + ": texcoords not 8-byte aligned");
            br[b].texcoords = reinterpret_cast<const float2 *>(tc.texcoords);
        }
        out.max_blas_depth = in.max_depth > out.max_blas_depth ? in.max_depth : out.max_blas_depth;
        if (in.n_tris > 0 && in.max_geom_id > out.max_geom_id) out.max_geom_id = in.max_geom_id;
    }
    for (uint32_t q = 0; q < n_inst; ++q) {
        if (instances[q].blas >= n_blas)
            return fail(RT_ERR_INVALID_ARG, "instance " + std::to_string(q) + ": blas out of range");
        ir[q].blas = instances[q].blas;
        for (int k = 0; k < 12; ++k) {
            if (!std::isfinite(instances[q].object_from_world[k]))
                return fail(RT_ERR_INVALID_ARG, "instance " + std::to_string(q) + ": non-finite map");
            ir[q].m[k] = instances[q].object_from_world[k];
        }
    }
    *info = out;
    g_last_error.clear();
    return RT_OK;
}

// Spill columns for the two-level stack (at most the top-level depth plus the
// deepest bottom-level BVH), one per ray.
static size_t instanced_workspace(const rt_bvh_info &tlas, uint32_t max_blas_depth, uint32_t n_rays)
{
    const uint32_t depth = tlas.max_depth + max_blas_depth;
    const uint32_t cap = kInstancedSlots - 1;
    const size_t threads = (size_t(n_rays) + 63) / 64 * 64;
    return size_t(depth > cap ? depth - cap : 0) * threads * sizeof(uint64_t);
}

static rt_status check_instance_info(const rt_instance_info *info)
{
    if (!info) return fail(RT_ERR_INVALID_ARG, "info is NULL");
    if (info->max_blas_depth >= 128) return fail(RT_ERR_INVALID_ARG, "max_blas_depth must be < 128");
    return RT_OK;
}

rt_status rt_trace_instanced_workspace_bytes(const rt_scene *tlas, const rt_instance_info *info,
                                             uint32_t n_rays, uint32_t flags, size_t *bytes)
{
    g_last_error.clear();
    if (!bytes) return fail(RT_ERR_INVALID_ARG, "bytes is NULL");
    rt_status st = check_scene(tlas);
    if (st != RT_OK) return st;
    if (tlas->info.layout != RT_LAYOUT_F32)
        return fail(RT_ERR_UNSUPPORTED, "instancing takes an RT_LAYOUT_F32 top-level scene");
    if (flags & ~(RT_FLAG_COUNT | RT_FLAG_TILE_MASK)) return fail(RT_ERR_UNSUPPORTED, "unknown flag bits");
    st = check_instance_info(info);
    if (st != RT_OK) return st;
    *bytes = instanced_workspace(tlas->info, info->max_blas_depth, n_rays);
    return RT_OK;
}

rt_status rt_trace_instanced(const rt_scene *tlas, const void *table, const rt_instance_info *info,
                             const rt_ray *rays, uint32_t n_rays, rt_isect_kind kind,
                             const void *params, uint32_t flags, int any_hit, void *out,
                             uint32_t *inst_ids, rt_counters *counters, void *workspace,
                             size_t workspace_bytes, void *stream)
{
    g_last_error.clear();
    rt_status st = check_scene(tlas);
    if (st != RT_OK) return st;
    if (tlas->info.layout != RT_LAYOUT_F32)
        return fail(RT_ERR_UNSUPPORTED, "instancing takes an RT_LAYOUT_F32 top-level scene");
    if (flags & ~(RT_FLAG_COUNT | RT_FLAG_TILE_MASK)) return fail(RT_ERR_UNSUPPORTED, "unknown flag bits");
    st = check_instance_info(info);
    if (st != RT_OK) return st;
    InstancedRequest q{};
    q.kind = kind;
    if (kind == RT_ISECT_PROCEDURAL) {
        if (!params) return fail(RT_ERR_INVALID_ARG, "procedural intersector needs rt_procedural_params");
        q.checker = *static_cast<const rt_procedural_params *>(params);
        if (q.checker.checker_n < 1 || q.checker.checker_n > 65536)
            return fail(RT_ERR_INVALID_ARG, "checker_n must be within 1..65536");
    } else if (kind == RT_ISECT_ALPHA) {
        if (!params) return fail(RT_ERR_INVALID_ARG, "alpha intersector needs rt_alpha_params");
        q.alpha = *static_cast<const rt_alpha_params *>(params);
        if (!info->has_texcoords)
            return fail(RT_ERR_INVALID_ARG, "the table was packed without texture coordinates");
        if (!q.alpha.textures || !aligned(q.alpha.textures, 4))
            return fail(RT_ERR_INVALID_ARG, "alpha textures NULL or misaligned");
        if (q.alpha.width < 1 || q.alpha.height < 1 || q.alpha.alpha_min > 255)
            return fail(RT_ERR_INVALID_ARG, "alpha texture size or alpha_min out of range");
        if (q.alpha.n_tex <= info->max_geom_id)
            return fail(RT_ERR_INVALID_ARG, "a mesh's geom_id exceeds the texture count");
        q.alpha.texcoords = nullptr;  // per mesh, from the table
    } else if (kind != RT_ISECT_DEFAULT) {
        return fail(RT_ERR_UNSUPPORTED, "unknown intersector kind");
    }
    if (n_rays == 0) return RT_OK;
    if (n_rays > RT_MAX_RAYS) return fail(RT_ERR_INVALID_ARG, "more than 2^31 rays in one call");
    if (!table || !aligned(table, 16)) return fail(RT_ERR_INVALID_ARG, "table NULL or not 16-byte aligned");
    if (!rays || !aligned(rays, 16)) return fail(RT_ERR_INVALID_ARG, "rays NULL or not 16-byte aligned");
    if (!out || !aligned(out, any_hit ? 4 : 16)) return fail(RT_ERR_INVALID_ARG, "output NULL or misaligned");
    if (inst_ids && !aligned(inst_ids, 4)) return fail(RT_ERR_MISALIGNED, "inst_ids not 4-byte aligned");
    const bool count = (flags & RT_FLAG_COUNT) != 0;
    if (count && (!counters || !aligned(counters, 16)))
        return fail(RT_ERR_INVALID_ARG, "RT_FLAG_COUNT needs a 16-byte aligned counters array");
    const size_t need = instanced_workspace(tlas->info, info->max_blas_depth, n_rays);
    if (need > 0 && (!workspace || workspace_bytes < need || !aligned(workspace, 16)))
        return fail(RT_ERR_WORKSPACE, "workspace smaller than rt_trace_instanced_workspace_bytes");
    q.tlas = tlas;
    q.table = table;
    q.rays = rays;
    q.n_rays = n_rays;
    q.count = count;
    q.any = any_hit != 0;
    q.out = out;
    q.inst_ids = inst_ids;
    q.counters = count ? counters : nullptr;
    q.spill = workspace;
    q.tile_w8 = (flags & RT_FLAG_TILE_MASK) >> RT_FLAG_TILE_SHIFT;
    q.stream = stream;
    const char *err = "";
    st = launch_instanced(q, &err);
    if (st != RT_OK) return fail(st, err);
    return RT_OK;
}

rt_status rt_trace_multi(const rt_scene *scene, const rt_ray *rays, uint32_t n_rays,
                         rt_isect_kind kind, const void *params, uint32_t flags, uint32_t k,
                         rt_hit *hits, uint32_t *n_hits, rt_counters *counters, void *workspace,
                         size_t workspace_bytes, void *stream)
{
    return trace_common(Query::Multi, scene, rays, n_rays, kind, params, flags, hits, 16,
                        counters, workspace, workspace_bytes, stream, k, n_hits);
}

rt_status rt_hit_backward(const rt_ray *rays, const rt_hit *hits, const float *grad_tuv,
                          uint32_t n_rays, const float *vertices, uint32_t n_vertices,
                          const uint32_t *faces, uint32_t n_tris, float *grad_vertices,
                          float *grad_rays, void *stream)
{
    g_last_error.clear();
    if (n_rays == 0) return RT_OK;
    if (n_rays > RT_MAX_RAYS) return fail(RT_ERR_INVALID_ARG, "more than 2^31 rays in one call");
    if (!rays || !hits || !grad_tuv) return fail(RT_ERR_INVALID_ARG, "rays/hits/grad_tuv are NULL");
    if (!aligned(rays, 16) || !aligned(hits, 16))
        return fail(RT_ERR_MISALIGNED, "rays and hits must be 16-byte aligned");
    if (!aligned(grad_tuv, 4)) return fail(RT_ERR_MISALIGNED, "grad_tuv not 4-byte aligned");
    if (n_tris > 0 && (!vertices || !faces || !grad_vertices))
        return fail(RT_ERR_INVALID_ARG, "vertices/faces/grad_vertices are NULL");
    if (!aligned(vertices, 4) || !aligned(faces, 4) || !aligned(grad_vertices, 4))
        return fail(RT_ERR_MISALIGNED, "vertex, face and gradient arrays must be 4-byte aligned");
    if (grad_rays && !aligned(grad_rays, 16))
        return fail(RT_ERR_MISALIGNED, "grad_rays not 16-byte aligned");
    BackwardRequest q;
    q.rays = rays;
    q.hits = hits;
    q.grad_tuv = grad_tuv;
    q.n_rays = n_rays;
    q.vertices = vertices;
    q.n_vertices = n_vertices;
    q.faces = faces;
    q.n_tris = n_tris;
    q.grad_vertices = grad_vertices;
    q.grad_rays = grad_rays;
    q.stream = stream;
    const char *err = "";
    const rt_status st = launch_hit_backward(q, &err);
    if (st != RT_OK) return fail(st, err);
    return RT_OK;
}

uint32_t rt_launch_shapes(uint32_t *blocks, uint32_t *lds_stacks, uint32_t *chunks,
                          uint32_t *queues, uint32_t cap)
{
    for (uint32_t i = 0; i < kNumShapes && i < cap; ++i) {
        if (blocks) blocks[i] = kShapes[i].block;
        if (lds_stacks) lds_stacks[i] = kShapes[i].lds_stack;
        if (chunks) chunks[i] = kShapes[i].chunk;
        if (queues) queues[i] = kShapes[i].queue;
    }
    return kNumShapes;
}

const char *rt_status_string(rt_status s)
{
    switch (s) {
    case RT_OK: return "RT_OK";
    case RT_ERR_INVALID_ARG: return "RT_ERR_INVALID_ARG";
    case RT_ERR_MISALIGNED: return "RT_ERR_MISALIGNED";
    case RT_ERR_UNSUPPORTED: return "RT_ERR_UNSUPPORTED";
    case RT_ERR_WORKSPACE: return "RT_ERR_WORKSPACE";
    case RT_ERR_HIP: return "RT_ERR_HIP";
    case RT_ERR_OUT_OF_MEMORY: return "RT_ERR_OUT_OF_MEMORY";
    }
    return "unknown rt_status";
}

const char *rt_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
