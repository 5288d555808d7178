// Layout of the scene table of a batched launch, shared by the host packer
// (C ABI) and the traversal kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace rtx {

// -------------------------------------------------------------------------
// batched launches: a device table of scenes, each owning a consecutive range
// of the batch's rays
//   [0, 64)                      header: n_scenes
//   [64, 64 + 4 (n_scenes + 1))  ray_begin prefix (uint32), padded to 64 B
//   then n_scenes records of 128 B (batch_scene below)
// -------------------------------------------------------------------------
struct alignas(16) batch_scene {
    const float4 *nodes;
    const float4 *tris;
    const float2 *texcoords;    // alpha-mask data of this scene (may be null)
    const uint32_t *textures;
    float root_lo[3], root_hi[3];
    uint32_t root_ref, n_tris;
    uint32_t tex_width, tex_height, alpha_min;
    uint32_t layout;            // RT_LAYOUT_F32, RT_LAYOUT_Q8 or RT_LAYOUT_WIDE4
    uint32_t pad[10];
};
static_assert(sizeof(batch_scene) == 128, "batch scene record");

__host__ __device__ constexpr size_t batch_prefix_offset() { return 64; }
__host__ __device__ constexpr size_t batch_records_offset(uint32_t n_scenes)
{
    return 64 + (size_t(n_scenes + 1) * 4 + 63) / 64 * 64;
}

// -------------------------------------------------------------------------
// instanced launches: a device table of bottom-level BVHs and instances
//   [0, 64)                        header: n_blas, n_inst
//   [64, 64 + 64 n_blas)           blas records (64 B)
//   then n_inst instance records (64 B)
// -------------------------------------------------------------------------
struct alignas(16) blas_record {
    const float4 *nodes;
    const float4 *tris;
    float root_lo[3], root_hi[3];
    uint32_t root_ref, n_tris;
    const float2 *texcoords;  // alpha mask: this mesh's texture coordinates
    uint32_t layout;          // RT_LAYOUT_F32 or RT_LAYOUT_Q8
    uint32_t pad;
};
static_assert(sizeof(blas_record) == 64, "blas record");

struct alignas(16) instance_record {
    uint32_t blas;
    uint32_t pad[3];
    float m[12];  // object_from_world, row-major 3x4
};
static_assert(sizeof(instance_record) == 64, "instance record");

__host__ __device__ constexpr size_t instance_blas_offset() { return 64; }
__host__ __device__ constexpr size_t instance_records_offset(uint32_t n_blas)
{
    return 64 + size_t(n_blas) * sizeof(blas_record);
}

}  // namespace rtx
