// Internal declarations shared by the host builder, the C ABI and the kernel
// launchers of librtx (not part of the public interface).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/rtx.h"

namespace rtx {

struct alignas(16) NodeRecord {
    union {
        float f[16];
        uint32_t u[16];
    };
};
static_assert(sizeof(NodeRecord) == RT_NODE_BYTES, "node record size");

struct alignas(16) TriRecord {
    union {
        float f[12];
        uint32_t u[12];
    };
};
static_assert(sizeof(TriRecord) == RT_TRI_BYTES, "triangle record size");

uint32_t max_inner_nodes(uint32_t n_tris);
rt_status build_bvh(const float *verts, const uint32_t *geom_ids, uint32_t n_tris,
                    NodeRecord *nodes, TriRecord *tris, rt_bvh_info *info);

enum class Query { Closest, Any };

// Launch shape of the traversal kernels: block size and on-chip stack depth.
struct LaunchShape {
    uint32_t block;      // threads per block
    uint32_t lds_stack;  // stack entries per lane held in LDS
};

// The shapes compiled into the library; the first one is the default.
extern const LaunchShape kShapes[];
extern const uint32_t kNumShapes;

struct TraceRequest {
    const rt_scene *scene;
    const void *rays;
    uint32_t n_rays;
    rt_isect_kind kind;
    rt_alpha_params alpha;
    rt_procedural_params checker;
    bool count;
    Query query;
    void *out;          // rt_hit* or uint32_t*
    void *counters;     // rt_counters* or null
    void *spill;        // workspace
    LaunchShape shape;
    void *stream;
};

// Spill entries per ray needed for a scene under a shape.
inline uint32_t spill_entries(const rt_bvh_info &info, const LaunchShape &s)
{
    return info.max_depth > s.lds_stack ? info.max_depth - s.lds_stack : 0u;
}

// Enqueues one traversal kernel; returns RT_OK or RT_ERR_HIP.
rt_status launch_trace(const TraceRequest &req, const char **err);

}  // namespace rtx
