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
// Two launches.  The first rewrites the triangle records (a lane per
// triangle) and zeroes one arrival counter per inner node.  The second gives
// each inner node a lane that writes the boxes of its leaf children into the
// node and adds their number to the node's counter; every inner child adds
// one when its own box is in place.  The lane whose addition completes a
// node's two children (the counter reaching 2) computes that node's box,
// writes it into the parent's slot (the host plan's parent words) and adds
// one there, and so on up; the root's completer writes the root box.  No
// lane waits: every other lane stops at its first incomplete node.  The
// additions are acquire-release at device scope, so a completer reads the
// slot its sibling's lane wrote before adding.
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

// Triangle records, and the counters zeroed (a lane per triangle or node).
__global__ __launch_bounds__(kRefitBlock) void refit_tris_kernel(TriRecord *tris, refit_mesh m,
                                                                 uint32_t *counters,
                                                                 uint32_t n_nodes)
{
    const uint32_t i = blockIdx.x * kRefitBlock + threadIdx.x;
    if (i < n_nodes) counters[i] = 0;
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

// Adds `arrivals` to node n's counter; true if that completes both children.
__device__ __forceinline__ bool arrive(uint32_t *counters, uint32_t n, uint32_t arrivals)
{
    const uint32_t before = __hip_atomic_fetch_add(counters + n, arrivals, __ATOMIC_ACQ_REL,
                                                   __HIP_MEMORY_SCOPE_AGENT);
    return before + arrivals == 2;
}

__global__ __launch_bounds__(kRefitBlock) void refit_nodes_kernel(NodeRecord *nodes,
                                                                  uint32_t n_nodes,
                                                                  const TriRecord *tris,
                                                                  const uint32_t *parents,
                                                                  uint32_t *counters, refit_mesh m,
                                                                  float *root_box)
{
    uint32_t n = blockIdx.x * kRefitBlock + threadIdx.x;
    if (n >= n_nodes) return;
    uint32_t leaves = 0;
    for (uint32_t c = 0; c < 2; ++c) {
        const uint32_t ref = nodes[n].u[12 + c];
        const uint32_t cnt = ref >> 29;
        if (cnt == 0) continue;
        float lo[3], hi[3];
        empty_box(lo, hi);
        grow_leaf(m, tris, ref & kRefIndexMaskHost, cnt, lo, hi);
        store_slot(nodes[n], c, lo, hi);
        ++leaves;
    }
    if (leaves == 0 || !arrive(counters, n, leaves)) return;
    // n's children are in place: climb while this lane completes nodes
    for (;;) {
        const NodeRecord &nd = nodes[n];
        const float l0[3] = {nd.f[0], nd.f[1], nd.f[2]}, h0[3] = {nd.f[3], nd.f[4], nd.f[5]};
        const float l1[3] = {nd.f[6], nd.f[7], nd.f[8]}, h1[3] = {nd.f[9], nd.f[10], nd.f[11]};
        float lo[3], hi[3];
        empty_box(lo, hi);
        grow(lo, hi, l0, h0);
        grow(lo, hi, l1, h1);
        const uint32_t up = parents[n];
        if (up == kRefitNoParent) {  // the root
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                root_box[a] = lo[a];
                root_box[3 + a] = hi[a];
            }
            return;
        }
        const uint32_t p = up >> 1;
        store_slot(nodes[p], up & 1u, lo, hi);
        if (!arrive(counters, p, 1)) return;
        n = p;
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
    const uint32_t lanes = q.n_tris > q.n_nodes ? q.n_tris : q.n_nodes;
    if (lanes > 0)
        hipLaunchKernelGGL(refit_tris_kernel, dim3((lanes + kRefitBlock - 1) / kRefitBlock),
                           dim3(kRefitBlock), 0, s, tris, m, q.counters, q.n_nodes);
    if (q.n_nodes > 0)
        hipLaunchKernelGGL(refit_nodes_kernel, dim3((q.n_nodes + kRefitBlock - 1) / kRefitBlock),
                           dim3(kRefitBlock), 0, s, nodes, q.n_nodes, tris, q.parents, q.counters,
                           m, q.root_box);
    else if (q.root_count > 0)
        hipLaunchKernelGGL(refit_root_leaf_kernel, dim3(1), dim3(64), 0, s, tris, q.root_first,
                           q.root_count, m, q.root_box);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        *err = hipGetErrorString(e);
        return RT_ERR_HIP;
    }
    return RT_OK;
}

}  // namespace rtx
