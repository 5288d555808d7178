// Refit of a built BVH (64-byte nodes) to new vertex positions: the tree's
// topology, node numbering and leaf order stay; the triangle records and
// every box are recomputed from an indexed mesh.
//
// Boxes grow from (+inf, -inf) by strict comparisons -- a lower bound moves
// only to a strictly smaller value, an upper bound only to a strictly larger
// one -- in a fixed order: a triangle's box over its vertices 0, 1, 2, a leaf
// child's over its triangles in leaf order, an inner child's over its own two
// child boxes (first, then second).  That is the order in which the builder
// grows a node's box over its triangles, so a refit to the build's vertices
// returns the build's boxes bit for bit, signs of zero included.  A vertex
// index past the mesh reads NaN, which no strict comparison accepts.
//
// Three launches, no atomics.  The first rewrites the triangle records (a
// lane per triangle).  In the second, block b owns the inner nodes numbered
// [256 b, 256 b + 256) (preorder numbers: a subtree is a contiguous range)
// and gives each a lane: every lane writes its node's leaf-child boxes, then,
// for depth d from the deepest to 0 with a block barrier between depths, the
// lanes whose node is at depth d and whose whole subtree lies in the block's
// range write their node's box into the parent's slot (or the root box).
// The nodes left -- "top" nodes, whose subtree leaves their block's range,
// listed by the host plan -- form the upper part of the tree; in the third
// launch one block finishes them the same way, depth by depth, their lower
// children being complete after the second launch.
#include <hip/hip_runtime.h>

#include <cmath>

#include "rt_internal.hpp"

namespace rtx {
namespace {

constexpr uint32_t kRefitBlock = 256;

struct refit_mesh {
    const float *vertices;  // [n_vertices][3]
    const uint32_t *faces;  // [n_tris][3] by input triangle index
    uint32_t n_vertices;
    uint32_t n_tris;
};

__device__ __forceinline__ void corner(const refit_mesh &m, uint32_t prim, int k, float p[3])
{
    const uint32_t vi = prim < m.n_tris ? m.faces[3 * size_t(prim) + k] : 0xFFFFFFFFu;
    if (vi < m.n_vertices) {
        p[0] = m.vertices[3 * size_t(vi)];
        p[1] = m.vertices[3 * size_t(vi) + 1];
        p[2] = m.vertices[3 * size_t(vi) + 2];
    } else {
        p[0] = p[1] = p[2] = __builtin_nanf("");
    }
}

__device__ __forceinline__ void grow(float lo[3], float hi[3], const float blo[3],
                                     const float bhi[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = blo[a] < lo[a] ? blo[a] : lo[a];
        hi[a] = bhi[a] > hi[a] ? bhi[a] : hi[a];
    }
}

__device__ __forceinline__ void empty_box(float lo[3], float hi[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = __builtin_inff();
        hi[a] = -__builtin_inff();
    }
}

// Grows (lo, hi) over the triangles [first, first + count) of the leaf order.
__device__ __forceinline__ void grow_leaf(const refit_mesh &m, const TriRecord *tris,
                                          uint32_t first, uint32_t count, float lo[3], float hi[3])
{
    for (uint32_t j = first; j < first + count; ++j) {
        const uint32_t prim = tris[j].u[3];
        for (int k = 0; k < 3; ++k) {
            float p[3];
            corner(m, prim, k, p);
            grow(lo, hi, p, p);
        }
    }
}

// Triangle records (a lane per triangle).
__global__ __launch_bounds__(kRefitBlock) void refit_tris_kernel(TriRecord *tris, refit_mesh m)
{
    const uint32_t i = blockIdx.x * kRefitBlock + threadIdx.x;
    if (i >= m.n_tris) return;
    TriRecord &t = tris[i];
    const uint32_t prim = t.u[3];
    float v0[3], v1[3], v2[3];
    corner(m, prim, 0, v0);
    corner(m, prim, 1, v1);
    corner(m, prim, 2, v2);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        t.f[a] = v0[a];
        t.f[4 + a] = v1[a] - v0[a];
        t.f[8 + a] = v2[a] - v0[a];
    }
}

__device__ __forceinline__ void store_slot(NodeRecord &nd, uint32_t c, const float lo[3],
                                           const float hi[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        nd.f[6 * c + a] = lo[a];
        nd.f[6 * c + 3 + a] = hi[a];
    }
}

// Node n's box from its two slots, written into its parent's slot (or, for
// the root, to root_box).
__device__ __forceinline__ void finish_node(NodeRecord *nodes, const uint32_t *parents,
                                            uint32_t n, float *root_box)
{
    const NodeRecord &nd = nodes[n];
    const float l0[3] = {nd.f[0], nd.f[1], nd.f[2]}, h0[3] = {nd.f[3], nd.f[4], nd.f[5]};
    const float l1[3] = {nd.f[6], nd.f[7], nd.f[8]}, h1[3] = {nd.f[9], nd.f[10], nd.f[11]};
    float lo[3], hi[3];
    empty_box(lo, hi);
    grow(lo, hi, l0, h0);
    grow(lo, hi, l1, h1);
    const uint32_t up = parents[n];
    if (up == kRefitNoParent) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            root_box[a] = lo[a];
            root_box[3 + a] = hi[a];
        }
        return;
    }
    store_slot(nodes[up >> 1], up & 1u, lo, hi);
}

static_assert(kRefitBlock == kRefitBlockNodes, "a refit block owns the plan's range of nodes");

__global__ __launch_bounds__(kRefitBlock) void refit_blocks_kernel(NodeRecord *nodes,
                                                                   uint32_t n_nodes,
                                                                   uint32_t max_depth,
                                                                   const TriRecord *tris,
                                                                   const uint32_t *plan,
                                                                   refit_mesh m, float *root_box)
{
    const uint32_t n = blockIdx.x * kRefitBlock + threadIdx.x;
    const bool mine = n < n_nodes;
    uint32_t depth_word = kRefitTopBit;
    if (mine) {
        depth_word = plan[n_nodes + n];
        for (uint32_t c = 0; c < 2; ++c) {
            const uint32_t ref = nodes[n].u[12 + c];
            const uint32_t cnt = ref >> 29;
            if (cnt == 0) continue;
            float lo[3], hi[3];
            empty_box(lo, hi);
            grow_leaf(m, tris, ref & kRefIndexMaskHost, cnt, lo, hi);
            store_slot(nodes[n], c, lo, hi);
        }
    }
    for (uint32_t d = max_depth + 1; d-- > 0;) {
        __syncthreads();
        if (depth_word == d) finish_node(nodes, plan, n, root_box);  // in range, not top
    }
}

// The top nodes, one block, depth by depth.
constexpr uint32_t kRefitTopBlock = 1024;
__global__ __launch_bounds__(kRefitTopBlock) void refit_top_kernel(NodeRecord *nodes,
                                                                   uint32_t n_nodes,
                                                                   uint32_t max_depth,
                                                                   const uint32_t *plan,
                                                                   uint32_t n_top, float *root_box)
{
    const uint32_t *top = plan + 2 * size_t(n_nodes);
    for (uint32_t d = max_depth + 1; d-- > 0;) {
        for (uint32_t i = threadIdx.x; i < n_top; i += kRefitTopBlock) {
            const uint32_t n = top[i];
            if ((plan[n_nodes + n] & ~kRefitTopBit) == d) finish_node(nodes, plan, n, root_box);
        }
        __syncthreads();
    }
}

// A root leaf: the root box over its triangles.
__global__ void refit_root_leaf_kernel(const TriRecord *tris, uint32_t first, uint32_t count,
                                       refit_mesh m, float *root_box)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float lo[3], hi[3];
    empty_box(lo, hi);
    grow_leaf(m, tris, first, count, lo, hi);
    for (int a = 0; a < 3; ++a) {
        root_box[a] = lo[a];
        root_box[3 + a] = hi[a];
    }
}

}  // namespace

rt_status launch_refit(const RefitRequest &q, const char **err)
{
    hipStream_t s = static_cast<hipStream_t>(q.stream);
    refit_mesh m{q.vertices, q.faces, q.n_vertices, q.n_tris};
    TriRecord *tris = static_cast<TriRecord *>(q.tris);
    NodeRecord *nodes = static_cast<NodeRecord *>(q.nodes);
    if (q.n_tris > 0)
        hipLaunchKernelGGL(refit_tris_kernel, dim3((q.n_tris + kRefitBlock - 1) / kRefitBlock),
                           dim3(kRefitBlock), 0, s, tris, m);
    if (q.n_nodes > 0) {
        hipLaunchKernelGGL(refit_blocks_kernel, dim3((q.n_nodes + kRefitBlock - 1) / kRefitBlock),
                           dim3(kRefitBlock), 0, s, nodes, q.n_nodes, q.max_depth, tris, q.plan, m,
                           q.root_box);
        if (q.n_top > 0)
            hipLaunchKernelGGL(refit_top_kernel, dim3(1), dim3(kRefitTopBlock), 0, s, nodes,
                               q.n_nodes, q.max_depth, q.plan, q.n_top, q.root_box);
    } else if (q.root_count > 0) {
        hipLaunchKernelGGL(refit_root_leaf_kernel, dim3(1), dim3(64), 0, s, tris, q.root_first,
                           q.root_count, m, q.root_box);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        *err = hipGetErrorString(e);
        return RT_ERR_HIP;
    }
    return RT_OK;
}

}  // namespace rtx
