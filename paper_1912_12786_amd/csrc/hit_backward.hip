// Adjoint of the accepted closest hit (differentiable hit).
//
// The hit point of a ray that hit triangle (v0, v1, v2) at (t, u, v) satisfies
// F = o + t d - (1-u-v) v0 - u v1 - v v2 = 0.  Differentiating implicitly
// with A = dF/d(t,u,v) = [d, -e1, -e2] gives, for an upstream gradient
// g = (dL/dt, dL/du, dL/dv), lam = -A^-T g and
//   dL/do = lam, dL/dd = t lam, dL/dv0 = -(1-u-v) lam, dL/dv1 = -u lam,
//   dL/dv2 = -v lam.
// A^T lam = -g is the 3x3 system d.lam = -g_t, e1.lam = g_u, e2.lam = g_v,
// solved with scalar triple products.  The hit prim and the intersector's
// accept decision are discrete and held fixed.
//
// One lane per ray; the per-ray algebra runs in float64 (half the float32
// vector rate on gfx950, ample for ~150 operations per ray) from the float32
// inputs.  Vertex gradients end in float32 hardware atomics (coarse-grained
// device memory), which are the kernel's cost, so they are merged first:
// neighbouring rays of a wave usually hit the same triangle, so each run of
// consecutive lanes with the same triangle sums its contributions (a
// segmented suffix scan over the wave); the runs' heads then add their three
// vertices' sums into a hash table in LDS keyed by vertex index, shared by
// the block's 1024 rays (two rows of a 512-wide image: neighbouring triangles
// share vertices), and one lane per table entry issues the three global
// atomics.  The summation order -- and the last bits of the sums -- vary from
// run to run.
#include <hip/hip_runtime.h>

#include "rt_internal.hpp"

namespace rtx {

constexpr uint32_t kNoPrim = 0xFFFFFFFFu;

struct backward_args {
    const float4 *rays;      // 2 float4 per ray
    const float4 *hits;      // (t, prim bits, u, v)
    const float *grad_tuv;   // [n][3]
    uint32_t n_rays;
    const float *vertices;   // [nv][3]
    uint32_t n_vertices;
    const uint32_t *faces;   // [n_tris][3]
    uint32_t n_tris;
    float *grad_vertices;    // [nv][3], accumulated
    float4 *grad_rays;       // [n][2] float4 or null
};

// Sums v over the lanes [lane, run_end] of the caller's run (run_end: last
// lane of the run, >= lane).  Every lane of the wave must call it.
__device__ __forceinline__ float run_suffix_sum(float v, uint32_t lane, uint32_t run_end)
{
#pragma unroll
    for (uint32_t off = 1; off < 64; off <<= 1) {
        const float w = __shfl_down(v, off, 64);
        if (lane + off <= run_end) v += w;
    }
    return v;
}

constexpr uint32_t kBackwardBlock = 1024;
constexpr uint32_t kTable = 4096;  // > 3 * kBackwardBlock keys, so probing always ends
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
static_assert((kTable & (kTable - 1)) == 0 && kTable > 3 * kBackwardBlock, "table size");

__global__ __launch_bounds__(kBackwardBlock) void hit_backward_kernel(backward_args a)
{
    __shared__ uint32_t tkey[kTable];
    __shared__ float tval[3][kTable];
    for (uint32_t s = threadIdx.x; s < kTable; s += kBackwardBlock) {
        tkey[s] = kEmpty;
        tval[0][s] = tval[1][s] = tval[2][s] = 0.0f;
    }
    const uint32_t i = blockIdx.x * kBackwardBlock + threadIdx.x;
    const bool in_range = i < a.n_rays;  // no early exit: the wave scans together
    uint32_t prim = kNoPrim;
    if (in_range) prim = __float_as_uint(a.hits[i].y);
    float lx = 0.0f, ly = 0.0f, lz = 0.0f;
    float tl[3] = {0.0f, 0.0f, 0.0f};  // t * lam
    float g[9] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};  // dL/dv0, dv1, dv2
    bool ok = in_range && prim < a.n_tris;
    uint32_t f0 = 0, f1 = 0, f2 = 0;
    if (ok) {
        f0 = a.faces[3 * size_t(prim)];
        f1 = a.faces[3 * size_t(prim) + 1];
        f2 = a.faces[3 * size_t(prim) + 2];
        ok = f0 < a.n_vertices && f1 < a.n_vertices && f2 < a.n_vertices;
    }
    if (ok) {
        // float64 evaluation from the float32 inputs: (t, u, v) of the fixed
        // triangle are recomputed (Moller-Trumbore), so that the gradient is
        // that of the exact hit of this triangle rather than of the float32
        // forward's rounded barycentrics
        const float4 r0 = a.rays[2 * size_t(i)];
        const float4 r1 = a.rays[2 * size_t(i) + 1];
        const double ox = r0.x, oy = r0.y, oz = r0.z;
        const double dx = r1.x, dy = r1.y, dz = r1.z;
        const float *p0 = a.vertices + 3 * size_t(f0);
        const float *p1 = a.vertices + 3 * size_t(f1);
        const float *p2 = a.vertices + 3 * size_t(f2);
        const double ax = p0[0], ay = p0[1], az = p0[2];
        const double e1x = double(p1[0]) - ax, e1y = double(p1[1]) - ay, e1z = double(p1[2]) - az;
        const double e2x = double(p2[0]) - ax, e2y = double(p2[1]) - ay, e2z = double(p2[2]) - az;
        // n = e1 x e2, c1 = e2 x d, c2 = d x e1 (c1 = -(d x e2))
        const double nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
        const double c1x = e2y * dz - e2z * dy, c1y = e2z * dx - e2x * dz, c1z = e2x * dy - e2y * dx;
        const double c2x = dy * e1z - dz * e1y, c2y = dz * e1x - dx * e1z, c2z = dx * e1y - dy * e1x;
        const double det = dx * nx + dy * ny + dz * nz;   // d.(e1 x e2)
        const double inv = 1.0 / det;
        const double sx = ox - ax, sy = oy - ay, sz = oz - az;
        // Cramer's rule on [d, -e1, -e2] (t, u, v) = v0 - o = -s with
        // det = d.(e1 x e2): u = s.(e2 x d) / det, v = -d.(s x e1) / det,
        // t = -e2.(s x e1) / det
        const double u = (sx * c1x + sy * c1y + sz * c1z) * inv;
        const double qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
        const double v = -(dx * qx + dy * qy + dz * qz) * inv;
        const double td = -(e2x * qx + e2y * qy + e2z * qz) * inv;
        const double gt = a.grad_tuv[3 * size_t(i)];
        const double gu = a.grad_tuv[3 * size_t(i) + 1];
        const double gv = a.grad_tuv[3 * size_t(i) + 2];
        const double lxd = (-gt * nx + gu * c1x + gv * c2x) * inv;
        const double lyd = (-gt * ny + gu * c1y + gv * c2y) * inv;
        const double lzd = (-gt * nz + gu * c1z + gv * c2z) * inv;
        const double w0 = (1.0 - u) - v;
        g[0] = float(-w0 * lxd);
        g[1] = float(-w0 * lyd);
        g[2] = float(-w0 * lzd);
        g[3] = float(-u * lxd);
        g[4] = float(-u * lyd);
        g[5] = float(-u * lzd);
        g[6] = float(-v * lxd);
        g[7] = float(-v * lyd);
        g[8] = float(-v * lzd);
        lx = float(lxd);
        ly = float(lyd);
        lz = float(lzd);
        tl[0] = float(td * lxd);
        tl[1] = float(td * lyd);
        tl[2] = float(td * lzd);
    }
    // runs of consecutive lanes with the same triangle (lanes without a valid
    // hit form runs of their own key and add nothing)
    const uint32_t lane = __lane_id();
    const uint32_t key = ok ? prim : kNoPrim;
    const uint32_t next_key = __shfl_down(key, 1, 64);
    const uint64_t tails = __ballot(lane == 63 || next_key != key);
    const uint32_t run_end = uint32_t(__ffsll((long long)(tails >> lane << lane)) - 1);
    const uint32_t prev_key = __shfl_up(key, 1, 64);
    const bool head = lane == 0 || prev_key != key;
#pragma unroll
    for (int k = 0; k < 9; ++k) g[k] = run_suffix_sum(g[k], lane, run_end);
    __syncthreads();  // the table is cleared
    if (ok && head) {
        const uint32_t fv[3] = {f0, f1, f2};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            // open addressing with linear probing: at most 3 * kBackwardBlock
            // keys in kTable slots, so an empty or matching slot is found
            uint32_t slot = (fv[k] * 2654435761u) >> 20;  // 12 bits: kTable = 4096
            for (;;) {
                const uint32_t old = atomicCAS(&tkey[slot], kEmpty, fv[k]);
                if (old == kEmpty || old == fv[k]) break;
                slot = (slot + 1) & (kTable - 1);
            }
            atomicAdd(&tval[0][slot], g[3 * k]);
            atomicAdd(&tval[1][slot], g[3 * k + 1]);
            atomicAdd(&tval[2][slot], g[3 * k + 2]);
        }
    }
    __syncthreads();
    for (uint32_t s = threadIdx.x; s < kTable; s += kBackwardBlock) {
        const uint32_t vtx = tkey[s];
        if (vtx == kEmpty) continue;
        float *gp = a.grad_vertices + 3 * size_t(vtx);
        unsafeAtomicAdd(gp + 0, tval[0][s]);
        unsafeAtomicAdd(gp + 1, tval[1][s]);
        unsafeAtomicAdd(gp + 2, tval[2][s]);
    }
    if (in_range && a.grad_rays) {
        a.grad_rays[2 * size_t(i)] = make_float4(lx, ly, lz, 0.0f);
        a.grad_rays[2 * size_t(i) + 1] = make_float4(tl[0], tl[1], tl[2], 0.0f);
    }
}

rt_status launch_hit_backward(const BackwardRequest &q, const char **err)
{
    backward_args a;
    a.rays = static_cast<const float4 *>(q.rays);
    a.hits = static_cast<const float4 *>(q.hits);
    a.grad_tuv = q.grad_tuv;
    a.n_rays = q.n_rays;
    a.vertices = q.vertices;
    a.n_vertices = q.n_vertices;
    a.faces = q.faces;
    a.n_tris = q.n_tris;
    a.grad_vertices = q.grad_vertices;
    a.grad_rays = static_cast<float4 *>(q.grad_rays);
    const uint32_t grid = (q.n_rays + kBackwardBlock - 1) / kBackwardBlock;
    hipLaunchKernelGGL(hit_backward_kernel, dim3(grid), dim3(kBackwardBlock), 0,
                       static_cast<hipStream_t>(q.stream), a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        *err = hipGetErrorString(e);
        return RT_ERR_HIP;
    }
    return RT_OK;
}

}  // namespace rtx
