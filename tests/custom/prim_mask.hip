// A user-defined intersector compiled into its own traversal kernels, the way
// an application injects one (Section 3.2: the intersector is a compile-time
// parameter of the traversal; Listing 3 shows a user intersector clearing
// hits).  This one keeps a hit iff the hit triangle's entry in a
// per-primitive byte mask is non-zero -- per-object visibility, a decision
// none of the library's built-in intersectors makes.
//
// Built by __graft_entry__.build() into tests/custom/libprim_mask.so; the GPU
// tests call it through the C functions below.
#include "../../paper_1912_12786_amd/csrc/rt_launch.hpp"

namespace {

struct prim_mask_intersector : rtx::intersector_base {
    static constexpr bool kFilters = true;
    struct params {
        const uint8_t *mask;  // device, [n_tris] by input triangle index
    };
    const uint8_t *mask;
    __device__ explicit prim_mask_intersector(const params &p) : mask(p.mask) {}
    __device__ __forceinline__ bool accept(const rtx::hit_candidate &c)
    {
        return mask[c.prim_id] != 0;
    }
};

thread_local const char *g_error = "";

}  // namespace

extern "C" {

// Workspace bytes for n_rays rays.
size_t prim_mask_workspace_bytes(const rt_scene *scene, uint32_t n_rays)
{
    return scene ? rtx::custom_workspace_bytes(*scene, n_rays) : 0;
}

// Closest hits keeping only triangles with mask[prim] != 0; with counters
// (non-NULL), also the four per-ray counts.  Returns an rt_status.
int prim_mask_trace(const rt_scene *scene, const rt_ray *rays, uint32_t n_rays,
                    const uint8_t *mask, rt_hit *hits, rt_counters *counters, void *workspace,
                    size_t workspace_bytes, void *stream)
{
    g_error = "";
    if (!mask && scene && scene->info.n_tris > 0) {
        g_error = "mask is NULL";
        return RT_ERR_INVALID_ARG;
    }
    const prim_mask_intersector::params p{mask};
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (counters)
        return rtx::trace_custom<rtx::counting_intersector<prim_mask_intersector>>(
            scene, rays, n_rays, p, hits, counters, workspace, workspace_bytes, s, &g_error);
    return rtx::trace_custom<prim_mask_intersector>(scene, rays, n_rays, p, hits, nullptr,
                                                   workspace, workspace_bytes, s, &g_error);
}

const char *prim_mask_last_error(void) { return g_error; }

}  // extern "C"
