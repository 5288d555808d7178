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
// One lane per triangle rewrites the records; then one launch per tree
// level, deepest first (the host plan from rt_bvh_refit_plan), gives each
// inner node of that level a lane that writes its two child boxes: a leaf
// child's from its triangles' vertices, an inner child's from the child's
// own record, written by the previous launch.
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

// The inner nodes order[first .. first + count) of one level: both child
// boxes; the root (node 0) also writes the root box.
__global__ __launch_bounds__(kRefitBlock) void refit_level_kernel(NodeRecord *nodes,
                                                                  const TriRecord *tris,
                                                                  const uint32_t *order,
                                                                  uint32_t first, uint32_t count,
                                                                  refit_mesh m, float *root_box)
{
    const uint32_t k = blockIdx.x * kRefitBlock + threadIdx.x;
    if (k >= count) return;
    const uint32_t n = order[first + k];
    NodeRecord &nd = nodes[n];
    float lo[2][3], hi[2][3];
    for (int c = 0; c < 2; ++c) {
        const uint32_t ref = nd.u[12 + c];
        const uint32_t cnt = ref >> 29, idx = ref & kRefIndexMaskHost;
        empty_box(lo[c], hi[c]);
        if (cnt) {
            grow_leaf(m, tris, idx, cnt, lo[c], hi[c]);
        } else {
            const NodeRecord &ch = nodes[idx];
            const float l0[3] = {ch.f[0], ch.f[1], ch.f[2]}, h0[3] = {ch.f[3], ch.f[4], ch.f[5]};
            const float l1[3] = {ch.f[6], ch.f[7], ch.f[8]}, h1[3] = {ch.f[9], ch.f[10], ch.f[11]};
            grow(lo[c], hi[c], l0, h0);
            grow(lo[c], hi[c], l1, h1);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        nd.f[a] = lo[0][a];
        nd.f[3 + a] = hi[0][a];
        nd.f[6 + a] = lo[1][a];
        nd.f[9 + a] = hi[1][a];
    }
    if (n == 0 && root_box) {
        float rlo[3], rhi[3];
        empty_box(rlo, rhi);
        grow(rlo, rhi, lo[0], hi[0]);
        grow(rlo, rhi, lo[1], hi[1]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            root_box[a] = rlo[a];
            root_box[3 + a] = rhi[a];
        }
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
    if (q.n_levels == 0) {  // a root leaf (or no triangles)
        if (q.root_count > 0 && q.root_box)
            hipLaunchKernelGGL(refit_root_leaf_kernel, dim3(1), dim3(64), 0, s, tris, q.root_first,
                               q.root_count, m, q.root_box);
    }
    for (uint32_t l = 0; l < q.n_levels; ++l) {
        const uint32_t first = q.level_start[l], count = q.level_start[l + 1] - first;
        if (count == 0) continue;
        hipLaunchKernelGGL(refit_level_kernel, dim3((count + kRefitBlock - 1) / kRefitBlock),
                           dim3(kRefitBlock), 0, s, nodes, tris, q.order, first, count, m,
                           q.root_box);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        *err = hipGetErrorString(e);
        return RT_ERR_HIP;
    }
    return RT_OK;
}

}  // namespace rtx
