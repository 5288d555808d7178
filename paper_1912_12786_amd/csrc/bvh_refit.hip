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
// Two launches, no atomics, every dependent step in LDS.  In the first,
// block b owns the inner nodes numbered [1024 b, 1024 b + 1024) (preorder
// numbers: a subtree is a contiguous range) and gives each a lane; the
// blocks after the nodes' rewrite the triangle records.  Every lane
// computes its node's leaf-child boxes; then, for depth d from the deepest to
// 0 with a block barrier between depths, the lanes whose node is at depth d
// and whose whole subtree lies in the block's range combine their two child
// boxes -- a leaf child's from registers, an inner child's from the block's
// LDS row of node boxes -- into their node's box in LDS.  Only then does
// each lane write its leaf-child slots and its node's box into the parent's
// slot (or the root box).  The nodes left -- "top" nodes, whose subtree
// leaves their block's range, listed by the host plan in increasing order --
// form the upper part of the tree, where a top node's parent is a top node
// too.  In the second launch one block loads their two slots into LDS (the
// lower children being final), finds each one's parent in the list by
// binary search, and finishes them depth by depth, each node writing its box
// into its parent's LDS slot; it writes the slots back at the end.  A list
// longer than that block's LDS is finished in global memory instead, the
// same way but one dependent load and store per depth.
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

__device__ __forceinline__ void refit_tri(TriRecord &t, const refit_mesh &m)
{
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

// The boxes of a node's leaf children (ref[c] with a count) over their
// triangles in leaf order, first child's into lb0, second's into lb1.  The
// triangles are gathered four at a time, so that their loads overlap, and
// each one's box (over its vertices 0, 1, 2) is grown into its child's: with
// strict comparisons that gives the bits of growing over the vertices one by
// one.
__device__ __forceinline__ void leaf_boxes(const refit_mesh &m, const TriRecord *tris,
                                           const uint32_t ref[2], float lb0[6], float lb1[6])
{
    const uint32_t c0 = ref[0] >> 29, c1 = ref[1] >> 29, total = c0 + c1;
    const uint32_t f0 = ref[0] & kRefIndexMaskHost, f1 = ref[1] & kRefIndexMaskHost;
    for (uint32_t e0 = 0; e0 < total; e0 += 4) {
        uint32_t prim[4];
#pragma unroll
        for (uint32_t s = 0; s < 4; ++s) {
            const uint32_t e = e0 + s;
            prim[s] = e < total ? tris[e < c0 ? f0 + e : f1 + (e - c0)].u[3] : 0xFFFFFFFFu;
        }
        float p[4][3][3];
#pragma unroll
        for (uint32_t s = 0; s < 4; ++s)
#pragma unroll
            for (int k = 0; k < 3; ++k) corner(m, prim[s], k, p[s][k]);
#pragma unroll
        for (uint32_t s = 0; s < 4; ++s) {
            const uint32_t e = e0 + s;
            if (e >= total) continue;
            float tlo[3], thi[3];
            empty_box(tlo, thi);
#pragma unroll
            for (int k = 0; k < 3; ++k) grow(tlo, thi, p[s][k], p[s][k]);
            if (e < c0) grow(lb0, lb0 + 3, tlo, thi);
            else grow(lb1, lb1 + 3, tlo, thi);
        }
    }
}

// Triangle records (a lane per triangle): a root leaf's scene, which has no
// inner nodes for the blocks kernel to carry them.
__global__ __launch_bounds__(kRefitBlock) void refit_tris_kernel(TriRecord *tris, refit_mesh m)
{
    const uint32_t i = blockIdx.x * kRefitBlock + threadIdx.x;
    if (i < m.n_tris) refit_tri(tris[i], m);
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

// A box into the parent's slot named by parent word up, or into root_box.
__device__ __forceinline__ void store_up(NodeRecord *nodes, uint32_t up, const float lo[3],
                                         const float hi[3], float *root_box)
{
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

// Node n's box from its two slots (global), written into its parent's slot.
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
    store_up(nodes, parents[n], lo, hi, root_box);
}

constexpr uint32_t kRefitNodesBlock = 1024;
static_assert(kRefitNodesBlock == kRefitBlockNodes, "a refit block owns the plan's range of nodes");

__global__ __launch_bounds__(kRefitNodesBlock) void refit_blocks_kernel(NodeRecord *nodes,
                                                                        uint32_t n_nodes,
                                                                        uint32_t node_blocks,
                                                                        uint32_t max_depth,
                                                                        TriRecord *tris,
                                                                        const uint32_t *plan,
                                                                        refit_mesh m,
                                                                        float *root_box)
{
    __shared__ float s_box[kRefitNodesBlock][6];
    if (blockIdx.x >= node_blocks) {  // the blocks after the nodes' rewrite the triangle records
        const size_t i = size_t(blockIdx.x - node_blocks) * kRefitNodesBlock + threadIdx.x;
        if (i < m.n_tris) refit_tri(tris[i], m);
        return;
    }
    const uint32_t base = blockIdx.x * kRefitNodesBlock;
    const uint32_t n = base + threadIdx.x;
    const bool mine = n < n_nodes;
    uint32_t depth_word = kRefitTopBit, ref[2] = {0u, 0u};
    float lb[2][6];
#pragma unroll
    for (uint32_t c = 0; c < 2; ++c) empty_box(lb[c], lb[c] + 3);
    if (mine) {
        depth_word = plan[n_nodes + n];
        ref[0] = nodes[n].u[12];
        ref[1] = nodes[n].u[13];
        leaf_boxes(m, tris, ref, lb[0], lb[1]);
    }
    // A node whose subtree lies in the block has its inner children in the
    // block too; an index outside (a plan of another tree) is skipped.
    for (uint32_t d = max_depth + 1; d-- > 0;) {
        __syncthreads();
        if (depth_word != d) continue;  // top nodes never match
        float lo[3], hi[3];
        empty_box(lo, hi);
#pragma unroll
        for (uint32_t c = 0; c < 2; ++c) {
            if ((ref[c] >> 29) != 0) {
                grow(lo, hi, lb[c], lb[c] + 3);
            } else {
                const uint32_t k = (ref[c] & kRefIndexMaskHost) - base;
                if (k < kRefitNodesBlock) grow(lo, hi, s_box[k], s_box[k] + 3);
            }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            s_box[threadIdx.x][a] = lo[a];
            s_box[threadIdx.x][3 + a] = hi[a];
        }
    }
    if (!mine) return;
#pragma unroll
    for (uint32_t c = 0; c < 2; ++c)
        if ((ref[c] >> 29) != 0) store_slot(nodes[n], c, lb[c], lb[c] + 3);
    if ((depth_word & kRefitTopBit) == 0)
        store_up(nodes, plan[n], s_box[threadIdx.x], s_box[threadIdx.x] + 3, root_box);
}

// The top nodes, one block.
constexpr uint32_t kRefitTopBlock = 1024;
constexpr uint32_t kRefitTopCap = 2048;          // top nodes the LDS version holds
static_assert(kRefitTopCap % kRefitTopBlock == 0, "whole entries per lane");
constexpr uint32_t kRefitLost = 0xFFFFFFFEu;     // a parent missing from the list

__global__ __launch_bounds__(kRefitTopBlock) void refit_top_lds_kernel(NodeRecord *nodes,
                                                                       uint32_t n_nodes,
                                                                       uint32_t max_depth,
                                                                       const uint32_t *plan,
                                                                       uint32_t n_top,
                                                                       float *root_box)
{
    // Lane t owns the list entries t and t + kRefitTopBlock: their node,
    // depth and parent link stay in registers; their slots sit in LDS, where
    // their children write.
    constexpr uint32_t kPer = kRefitTopCap / kRefitTopBlock;
    __shared__ uint32_t s_id[kRefitTopCap];
    __shared__ float s_slot[kRefitTopCap][12];  // the node's two child boxes
    const uint32_t *top = plan + 2 * size_t(n_nodes);
    uint32_t id[kPer], depth[kPer], link[kPer];
#pragma unroll
    for (uint32_t r = 0; r < kPer; ++r) {
        const uint32_t i = threadIdx.x + r * kRefitTopBlock;
        id[r] = i < n_top ? top[i] : kRefitNoParent;
        if (i < n_top) s_id[i] = id[r];
    }
    __syncthreads();
#pragma unroll
    for (uint32_t r = 0; r < kPer; ++r) {
        const uint32_t i = threadIdx.x + r * kRefitTopBlock;
        depth[r] = kRefitNoParent;
        link[r] = kRefitLost;
        if (id[r] >= n_nodes) continue;  // past the list, or a plan of another tree
        const NodeRecord &nd = nodes[id[r]];
#pragma unroll
        for (int a = 0; a < 12; ++a) s_slot[i][a] = nd.f[a];
        depth[r] = plan[n_nodes + id[r]] & ~kRefitTopBit;
        const uint32_t up = plan[id[r]];
        if (up == kRefitNoParent) {
            link[r] = kRefitNoParent;
            continue;
        }
        const uint32_t p = up >> 1;
        uint32_t lo = 0, hi = n_top;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_id[mid] < p) lo = mid + 1;
            else hi = mid;
        }
        if (lo < n_top && s_id[lo] == p) link[r] = (lo << 1) | (up & 1u);
    }
    // A node at depth d reads its own slots and writes its parent's (depth
    // d - 1), so the barrier between depths orders every read after the
    // writes it needs.
    for (uint32_t d = max_depth + 1; d-- > 0;) {
        __syncthreads();
#pragma unroll
        for (uint32_t r = 0; r < kPer; ++r) {
            if (depth[r] != d) continue;
            const float *sl = s_slot[threadIdx.x + r * kRefitTopBlock];
            float lo[3], hi[3];
            empty_box(lo, hi);
            grow(lo, hi, sl, sl + 3);
            grow(lo, hi, sl + 6, sl + 9);
            if (link[r] == kRefitNoParent) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    root_box[a] = lo[a];
                    root_box[3 + a] = hi[a];
                }
            } else if (link[r] != kRefitLost) {
                float *ps = s_slot[link[r] >> 1] + 6 * (link[r] & 1u);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    ps[a] = lo[a];
                    ps[3 + a] = hi[a];
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (uint32_t r = 0; r < kPer; ++r) {
        if (id[r] >= n_nodes) continue;
        NodeRecord &nd = nodes[id[r]];
        const float *sl = s_slot[threadIdx.x + r * kRefitTopBlock];
#pragma unroll
        for (int a = 0; a < 12; ++a) nd.f[a] = sl[a];
    }
}

// More top nodes than the LDS version holds: depth by depth in global
// memory, each node's box read from its slots and written into its parent's.
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
            if (n < n_nodes && (plan[n_nodes + n] & ~kRefitTopBit) == d)
                finish_node(nodes, plan, n, root_box);
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
    if (q.n_nodes > 0) {
        const uint32_t node_blocks = (q.n_nodes + kRefitNodesBlock - 1) / kRefitNodesBlock;
        const uint32_t tri_blocks = (q.n_tris + kRefitNodesBlock - 1) / kRefitNodesBlock;
        hipLaunchKernelGGL(refit_blocks_kernel, dim3(node_blocks + tri_blocks),
                           dim3(kRefitNodesBlock), 0, s, nodes, q.n_nodes, node_blocks, q.max_depth,
                           tris, q.plan, m, q.root_box);
        if (q.n_top > kRefitTopCap)
            hipLaunchKernelGGL(refit_top_kernel, dim3(1), dim3(kRefitTopBlock), 0, s, nodes,
                               q.n_nodes, q.max_depth, q.plan, q.n_top, q.root_box);
        else if (q.n_top > 0)
            hipLaunchKernelGGL(refit_top_lds_kernel, dim3(1), dim3(kRefitTopBlock), 0, s, nodes,
                               q.n_nodes, q.max_depth, q.plan, q.n_top, q.root_box);
    } else {
        if (q.n_tris > 0)
            hipLaunchKernelGGL(refit_tris_kernel, dim3((q.n_tris + kRefitBlock - 1) / kRefitBlock),
                               dim3(kRefitBlock), 0, s, tris, m);
        if (q.root_count > 0)
            hipLaunchKernelGGL(refit_root_leaf_kernel, dim3(1), dim3(64), 0, s, tris,
                               q.root_first, q.root_count, m, q.root_box);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        *err = hipGetErrorString(e);
        return RT_ERR_HIP;
    }
    return RT_OK;
}

}  // namespace rtx
