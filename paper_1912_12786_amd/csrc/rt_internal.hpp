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

struct alignas(16) NodeQ8Record {
    uint32_t u[8];
};
static_assert(sizeof(NodeQ8Record) == RT_NODE_BYTES_Q8, "compressed node record size");

struct alignas(16) NodePackedRecord {
    uint32_t u[12];
};
static_assert(sizeof(NodePackedRecord) == RT_NODE_BYTES_F32P, "packed node record size");

struct alignas(16) NodeW4Record {
    union {
        float f[32];
        uint32_t u[32];
    };
};
static_assert(sizeof(NodeW4Record) == RT_NODE_BYTES_WIDE4, "four-wide node record size");

constexpr uint32_t kRefIndexMaskHost = 0x1FFFFFFFu;

// Inner nodes of a BVH over n_tris triangles with leaves of at most max_leaf.
uint32_t max_inner_nodes(uint32_t n_tris, uint32_t max_leaf);
rt_status build_bvh(const float *verts, const uint32_t *geom_ids, uint32_t n_tris,
                    uint32_t max_leaf, NodeRecord *nodes, TriRecord *tris, rt_bvh_info *info);
// 64-B nodes -> 32-B nodes (RT_ERR_INVALID_ARG if a box is not finite).
rt_status compress_nodes(const NodeRecord *in, uint32_t n_nodes, NodeQ8Record *out);
// 64-B nodes -> 48-B nodes carrying their references in moved box words
// (RT_ERR_INVALID_ARG if a box is not finite or a word cannot move).
rt_status pack_nodes(const NodeRecord *in, uint32_t n_nodes, NodePackedRecord *out);
// 64-B binary nodes -> 128-B four-wide nodes (at most info.n_nodes of them);
// RT_ERR_INVALID_ARG if a child reference is out of range.
rt_status widen_nodes(const NodeRecord *in, const rt_bvh_info &info, NodeW4Record *out,
                      uint32_t *n_out, uint32_t *stack_bound);

enum class Query { Closest, Any, Multi };

// Launch shape of the traversal kernels.
struct LaunchShape {
    uint32_t block;      // threads per block
    uint32_t lds_stack;  // LDS ring slots per lane (holds lds_stack - 1 stack entries)
    uint32_t chunk;      // rays a wave takes at a time (its lanes refill from them)
    uint32_t queue;      // 1: persistent grid + global atomic ray queue; 0: static chunks
};

// Waves of a persistent (queue) grid: 256 CUs x 32 wave slots of MI355X.
// Surplus waves of a lower-occupancy kernel start late, find the queue
// drained and exit.
constexpr uint64_t kPersistentWaves = 256 * 32;

// Workspace layout: the queue heads in the first 1024 bytes (queue shapes:
// 8 heads, 128 bytes apart), then the spill columns.
constexpr size_t kQueueBytes = 1024;

// The shapes compiled into the library; the first one is the default.
constexpr LaunchShape kDefaultShape{64, 8, 64, 1};
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
    void *out;          // rt_hit* (multi: [n][multi_k]) or uint32_t*
    void *n_hits;       // multi-hit: uint32_t* kept hits per ray
    uint32_t multi_k;   // multi-hit: hits kept per ray (1..RT_MAX_MULTI)
    void *counters;     // rt_counters* or null
    const void *batch;  // batched launch: device scene table (closest query), else null
    uint32_t runtime_dispatch;  // 0: compile-time intersector; 1: runtime switch; 2: indirect call
    void *spill;        // workspace past the queue head
    void *queue;        // queue head (queue shapes)
    LaunchShape shape;
    uint32_t tile_w8;   // tiled schedule: image width / 8 (0: index order)
    void *order;        // longest-path-first: the chunk-order area (else null)
    uint32_t waves_per_simd;  // queue shapes: most resident waves per SIMD (1..15)
    void *stream;
};

// Stack entries per lane that may have to live in global memory: the stack
// never holds more than max_depth entries and the ring keeps lds_stack - 1.
inline uint32_t spill_entries(const rt_bvh_info &info, const LaunchShape &s)
{
    const uint32_t cap = s.lds_stack - 1;
    return info.max_depth > cap ? info.max_depth - cap : 0u;
}

// Threads launched for n_rays rays (one column of spill space each).
inline uint64_t launch_threads(uint32_t n_rays, const LaunchShape &s)
{
    // one wave per chunk; a queue grid at most fills the chip
    uint64_t waves = (uint64_t(n_rays) + s.chunk - 1) / s.chunk;
    if (s.queue && waves > kPersistentWaves) waves = kPersistentWaves;
    return (waves * 64 + s.block - 1) / s.block * s.block;
}

// Workspace bytes of a single-scene launch of n_rays rays in shape s.
// Chunk-order area of a longest-path-first launch: a key and an order entry
// per chunk (chunks of s.chunk rays), then one row of kOrderAreaBuckets
// counts for each kOrderAreaRowChunks chunks (the keying kernel's per-block
// tallies; the kernels assert the same two numbers).
constexpr size_t kOrderAreaBuckets = 64;
constexpr size_t kOrderAreaRowChunks = 256;
inline size_t order_bytes(uint32_t n_rays, const LaunchShape &s)
{
    const size_t n_chunks = (size_t(n_rays) + s.chunk - 1) / s.chunk;
    const size_t n_rows = (n_chunks + kOrderAreaRowChunks - 1) / kOrderAreaRowChunks;
    return (8 * n_chunks + 4 * kOrderAreaBuckets * n_rows + 15) / 16 * 16;
}

inline size_t workspace_for(const rt_bvh_info &info, uint32_t n_rays, const LaunchShape &s,
                            bool longest_first = false)
{
    return (s.queue ? kQueueBytes : 0) + (longest_first ? order_bytes(n_rays, s) : 0) +
           size_t(spill_entries(info, s)) * size_t(launch_threads(n_rays, s)) * sizeof(uint64_t);
}

// Enqueues one traversal kernel; returns RT_OK or RT_ERR_HIP.
rt_status launch_trace(const TraceRequest &req, const char **err);

struct InstancedRequest {
    const rt_scene *tlas;
    const void *table;     // device instance table
    const void *rays;
    uint32_t n_rays;
    rt_isect_kind kind;
    rt_procedural_params checker;
    rt_alpha_params alpha;  // textures for every mesh (texcoords per mesh)
    bool count, any;
    void *out;             // rt_hit* or uint32_t* (any)
    uint32_t *inst_ids;    // may be null
    void *counters;
    void *spill;
    uint32_t tile_w8;      // tiled schedule: image width / 8 (0: index order)
    void *stream;
};

// Refit plan of a built BVH, 3 * n_nodes words at most:
//   [0, n)        parent words: 2 * (k's parent) + (k's slot in it) for every
//                 inner node k but the root, kRefitNoParent for the root;
//   [n, 2n)       depth of node k, | kRefitTopBit if k's subtree (the
//                 preorder range [k, k + size)) leaves the range of
//                 kRefitBlockNodes numbers that k's block of the refit owns;
//   [2n, 2n + t)  the t such "top" nodes.
// Returns t, or UINT32_MAX if a child reference is not a later node or a
// node is not the child of exactly one node.
constexpr uint32_t kRefitNoParent = 0xFFFFFFFFu;
constexpr uint32_t kRefitTopBit = 0x80000000u;
constexpr uint32_t kRefitBlockNodes = 1024;
uint32_t refit_plan(const NodeRecord *nodes, const rt_bvh_info &info, uint32_t *plan);

struct RefitRequest {
    void *nodes;              // device, n_nodes 64-byte records (rewritten)
    uint32_t n_nodes;
    uint32_t max_depth;       // deepest inner node's depth bound (the tree's max_depth)
    void *tris;               // device, n_tris triangle records (rewritten)
    uint32_t n_tris;
    const uint32_t *plan;     // device, the plan (2 * n_nodes + n_top words)
    uint32_t n_top;
    uint32_t root_first, root_count;  // a root leaf's triangles (n_nodes == 0)
    const float *vertices;    // device [n_vertices][3]
    uint32_t n_vertices;
    const uint32_t *faces;    // device [n_tris][3]
    float *root_box;          // device, 6 floats out
    void *stream;
};
rt_status launch_refit(const RefitRequest &req, const char **err);

// Instanced traversal: one ray per lane, one wave per 64 consecutive rays (no
// refill: rays of a wave stay coherent, so its lanes tend to enter the same
// instances together), LDS ring of kInstancedSlots.
constexpr uint32_t kInstancedSlots = 8;
rt_status launch_instanced(const InstancedRequest &req, const char **err);

struct BackwardRequest {
    const void *rays;
    const void *hits;
    const float *grad_tuv;
    uint32_t n_rays;
    const float *vertices;
    uint32_t n_vertices;
    const uint32_t *faces;
    uint32_t n_tris;
    float *grad_vertices;
    void *grad_rays;
    void *stream;
};

// Enqueues the adjoint of the accepted hits; returns RT_OK or RT_ERR_HIP.
rt_status launch_hit_backward(const BackwardRequest &req, const char **err);

}  // namespace rtx
