/*
 * rtx.h -- C ABI of librtx: BVH ray traversal with compile-time custom
 * intersectors on AMD Instinct MI355X (gfx950).
 *
 * The operations follow Section 3.1 of Zellmann, "Adding Custom Intersectors
 * to the C++ Ray Tracing Template Library Visionaray" (2019):
 *   - closest_hit(ray, prims, intersector): the nearest hit point that the
 *     intersector accepts;
 *   - any_hit(ray, prims, intersector): the first accepted hit encountered;
 *   - an intersector is a compile-time type that intercepts the ray/box and
 *     ray/primitive tests of the traversal (Section 3.2, Algorithm 1) and may
 *     clear a hit (Listing 3); the use cases of Section 4 are built in:
 *     alpha mask (Listing 5), procedural alpha mask, and the BVH-cost counter
 *     (Listing 6).
 * A C ABI cannot take a template, so every built-in intersector x query x
 * counting combination is a separate kernel instantiation compiled into the
 * library, and the host selects one per launch.  C++/HIP code can instead
 * include rt_traverse.hpp and instantiate the traversal with its own functor.
 *
 * Conventions
 *   - Every pointer marked "device" is device memory owned by the caller;
 *     every pointer marked "host" is host memory owned by the caller.  The
 *     library never allocates device memory and never frees anything.
 *   - Device arrays of rays, hits, counters, nodes and triangle records must
 *     be 16-byte aligned.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).  Trace
 *     calls only enqueue work; device faults surface at the caller's next
 *     synchronisation.
 *   - Every entry point returns an rt_status; on failure nothing is enqueued
 *     and rt_last_error() describes the reason (thread-local).
 *   - Ray components must be finite and tmin <= tmax (tmax may be +inf);
 *     other rays give unspecified (but memory-safe) results.
 */
#ifndef RTX_H
#define RTX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rt_status {
    RT_OK = 0,
    RT_ERR_INVALID_ARG = -1,  /* null pointer, bad size, inconsistent scene */
    RT_ERR_MISALIGNED = -2,   /* a device array is not 16-byte aligned */
    RT_ERR_UNSUPPORTED = -3,  /* unknown intersector kind or flag; combination not compiled in */
    RT_ERR_WORKSPACE = -4,    /* workspace missing or smaller than required */
    RT_ERR_HIP = -5,          /* a HIP runtime call failed */
    RT_ERR_OUT_OF_MEMORY = -6 /* host scratch allocation in the builder failed */
} rt_status;

/* A ray o + t d, valid for tmin < t < tmax (both ends excluded). 32 bytes. */
typedef struct rt_ray {
    float ox, oy, oz, tmin;
    float dx, dy, dz, tmax;
} rt_ray;

/* Closest-hit record (the paper's hit_record: distance t, prim_id, and the
 * barycentrics u, v with P = (1-u-v) v0 + u v1 + v v2).  prim_id is the index
 * of the triangle in the caller's input array.  A miss has
 * prim_id = RT_MISS, t = +inf, u = v = 0.  16 bytes. */
typedef struct rt_hit {
    float t;
    uint32_t prim_id;
    float u, v;
} rt_hit;

#define RT_MISS 0xFFFFFFFFu

/* Per-ray counts of the heat-map intersector (Section 4, Listing 6):
 * num_boxes  -- ray/box tests executed (root box + 2 per inner node entered),
 * num_tris   -- ray/triangle tests executed, misses included,
 * num_candidates -- geometric hits inside the current interval that were
 *               handed to the intersector's accept decision,
 * num_accepted   -- candidates the intersector accepted.  16 bytes. */
typedef struct rt_counters {
    uint32_t num_boxes, num_tris, num_candidates, num_accepted;
} rt_counters;

typedef enum rt_isect_kind {
    RT_ISECT_DEFAULT = 0,    /* accept every hit; compiled to no code at all */
    RT_ISECT_ALPHA = 1,      /* alpha mask: params = const rt_alpha_params*    */
    RT_ISECT_PROCEDURAL = 2  /* checker mask: params = const rt_procedural_params* */
} rt_isect_kind;

/* Flags.  RT_FLAG_COUNT composes the counting intersector with the chosen
 * kind and requires a counters array.
 * RT_FLAG_RUNTIME_SWITCH / RT_FLAG_RUNTIME_CALL (closest-hit query, without
 * counting) select the intersector per candidate at run time instead of at
 * compile time -- an inlined switch over the kinds, or an indirect call
 * through a table of filter functions, the way a library without templates
 * must do it (Section 1).  Results are identical; they exist to measure the
 * cost that compile-time injection avoids. */
#define RT_FLAG_COUNT 0x1u
#define RT_FLAG_RUNTIME_SWITCH 0x2u
#define RT_FLAG_RUNTIME_CALL 0x4u

/* Longest-path-first schedule: before the traversal, the rays are grouped in
 * the chunks that lanes take (64 rays in the default launch shape: tiles of
 * the tiled schedule, or runs of consecutive rays), each chunk is keyed by
 * the longest stretch inside the scene box of the intervals [tmin, tmax] of
 * four of its rays, the ends of its first and last runs of 8 (the corners of
 * an 8 x 8 tile), in 64 steps of the box diagonal, and the chunks are handed
 * out in decreasing key order.  A ray's work grows with the length of scene it crosses, and the
 * launch ends when its last and longest rays do, so starting the long ones
 * first shortens the tail.  Only the schedule changes: every ray's result,
 * counters and output position are those of the call without it.  The
 * workspace grows by 8 bytes per chunk plus 256 bytes per 256 chunks (or
 * part), rounded up to 16 (rt_trace_workspace_bytes with the same flags);
 * single-scene calls only (RT_ERR_UNSUPPORTED for batches). */
#define RT_FLAG_LONGEST_FIRST 0x8u

/* Launch shape of one call: bits 8..15 of flags hold an index into the table
 * that rt_launch_shapes lists (0, the default, when the field is clear).  The
 * shape is chosen per call, so calls on different threads or streams may use
 * different shapes; the workspace queries take the same flags, because the
 * workspace size depends on the shape.  Results never depend on the shape.
 * An index past the table is RT_ERR_UNSUPPORTED. */
#define RT_FLAG_SHAPE_SHIFT 8u
#define RT_FLAG_SHAPE_MASK 0xFF00u
#define RT_FLAG_SHAPE(index) ((((uint32_t)(index)) << RT_FLAG_SHAPE_SHIFT) & RT_FLAG_SHAPE_MASK)

/* Tiled schedule (a hint for rays that form an image in scanline order, such
 * as a camera's primary rays): bits 16..27 of flags hold W/8 for an image W
 * pixels wide (W a multiple of 8, at most 32760).  Rays are then handed to the
 * GPU's lanes in 8 x 8 pixel tiles instead of in index order: the first
 * 8 * W * floor(n_rays / (8 W)) rays (whole rows of tiles) are taken tile by
 * tile, the rest in index order.  Only which lanes trace which rays, and
 * when, changes: every ray's result and counters, and where they are written
 * (at the ray's index), are those of the untiled call.  Single-scene calls
 * (rt_trace_closest, rt_trace_closest_noalloc, rt_trace_any, rt_trace_multi)
 * and rt_trace_instanced (one wave per tile) take it; an image wider than
 * 32760 is RT_ERR_INVALID_ARG. */
#define RT_FLAG_TILE_SHIFT 16u
#define RT_FLAG_TILE_MASK 0x0FFF0000u
#define RT_FLAG_TILE_WIDTH(width) ((((uint32_t)(width) / 8u) << RT_FLAG_TILE_SHIFT) & RT_FLAG_TILE_MASK)

/* Persistent-grid size, and so rays per lane, of launch shapes with a queue:
 * bits 28..31 of flags hold W, the most waves per SIMD the launch keeps
 * resident (1..15; 0 selects RT_DEFAULT_WAVES_PER_SIMD).  A queue launch
 * puts min(W, what the kernel's registers and LDS allow) waves on each of a
 * CU's 4 SIMDs (at least one block per CU), and its lanes take rays until the
 * queue drains, so each lane traces n_rays / (64 x the grid's waves) rays on
 * average.  Fewer resident waves keep fewer rays' node paths in a CU's
 * caches at once.  Results and counters never depend on W; shapes without a
 * queue (one lane per ray) ignore it.  Every entry point that takes flags
 * takes it. */
#define RT_FLAG_WAVES_SHIFT 28u
#define RT_FLAG_WAVES_MASK 0xF0000000u
#define RT_FLAG_WAVES_PER_SIMD(w) ((((uint32_t)(w)) << RT_FLAG_WAVES_SHIFT) & RT_FLAG_WAVES_MASK)
#define RT_DEFAULT_WAVES_PER_SIMD 7u

/* Alpha-mask intersector (Listing 5).  For a candidate (prim, u, v):
 *   (s, t) = (1-u-v) tc[prim][0] + u tc[prim][1] + v tc[prim][2],
 *   texel  = nearest texel (clamp to edge) of texture geom_id(prim),
 *   accept iff (texel >> 24) >= alpha_min.
 * A float threshold tau on alpha/255 is alpha_min = ceil(255 tau). */
typedef struct rt_alpha_params {
    const float *texcoords;     /* device, [n_texcoord_prims][3][2] by input triangle index */
    const uint32_t *textures;   /* device, [n_tex][height][width] RGBA8, R in the low byte */
    uint32_t n_texcoord_prims;  /* must be >= the scene's n_tris */
    uint32_t n_tex;             /* must be > the scene's max_geom_id */
    uint32_t width, height;     /* texel dimensions, each >= 1 */
    uint32_t alpha_min;         /* 0..255 */
} rt_alpha_params;

/* Procedural intersector: accept iff floor(n u) + floor(n v) is even. */
typedef struct rt_procedural_params {
    uint32_t checker_n;         /* >= 1 */
} rt_procedural_params;

/* Inner-node layouts (rt_bvh_info.layout). */
#define RT_LAYOUT_F32 0u  /* 64-B nodes with float32 child boxes (rt_bvh_build) */
#define RT_LAYOUT_Q8 1u   /* 32-B nodes with 8-bit child boxes (rt_bvh_compress) */
#define RT_LAYOUT_WIDE4 2u /* 128-B nodes with up to four float32 child boxes (rt_bvh_widen) */
#define RT_LAYOUT_F32P 3u  /* 48-B nodes, float32 child boxes carrying the child references (rt_bvh_pack) */

/* Description of a built BVH (filled by rt_bvh_build). */
typedef struct rt_bvh_info {
    uint32_t n_tris;
    uint32_t n_nodes;        /* inner nodes written (0 when the root is a leaf) */
    uint32_t max_depth;      /* deepest node; the traversal stack never exceeds it */
    uint32_t max_geom_id;
    uint32_t root_ref;       /* packed reference of the root item */
    float root_lo[3], root_hi[3];
    uint32_t layout;         /* RT_LAYOUT_F32, RT_LAYOUT_Q8 or RT_LAYOUT_WIDE4 */
    uint32_t max_leaf;       /* leaf size limit the BVH was built with (0 is read as 4) */
} rt_bvh_info;

/* A built BVH resident in device memory: a non-owning view.  nodes and tris
 * must be copies of what rt_bvh_build (and rt_bvh_compress for
 * RT_LAYOUT_Q8) wrote (the kernels follow the child references without
 * bounds checks; only the root is validated). */
typedef struct rt_scene {
    const void *nodes;       /* device, n_nodes records of the layout's size (RT_NODE_BYTES*) */
    const void *tris;        /* device, n_tris records of RT_TRI_BYTES */
    rt_bvh_info info;
} rt_scene;

#define RT_NODE_BYTES 64u
#define RT_NODE_BYTES_Q8 32u
#define RT_NODE_BYTES_WIDE4 128u
#define RT_NODE_BYTES_F32P 48u
#define RT_WIDE_EMPTY_REF 0xFFFFFFFFu  /* reference of an unused four-wide child slot */
#define RT_TRI_BYTES 48u
#define RT_MAX_TRIS 0x1FFFFFFFu  /* 2^29 - 1 */
#define RT_MAX_RAYS 0x80000000u  /* rays per trace call */

/* Upper bounds of the host buffers rt_bvh_build writes for n_tris triangles
 * (BVH construction is not described in the paper -- Section 3.1 only says
 * the BVH is built over the primitives -- so the builder is this library's:
 * binned surface-area heuristic, see rt_bvh_build).  The bounds hold for any
 * leaf size of rt_bvh_build_ex. */
rt_status rt_bvh_buffer_bytes(uint32_t n_tris, size_t *node_bytes, size_t *tri_bytes);

/* Builds the BVH on the host.
 *   vertices  host, [n_tris][3][3] float (triangle, corner, xyz)
 *   geom_ids  host, [n_tris] uint32 or NULL (all 0); used by the alpha mask
 *   nodes     host output, capacity node_cap bytes (rt_bvh_buffer_bytes)
 *   tris      host output, capacity tri_cap bytes
 *   info      host output
 * Construction: leaves hold at most 4 triangles (rt_bvh_build_ex: max_leaf); a
 * larger node is split at the
 * cheapest of 32 equal-width centroid bins per axis (surface-area cost,
 * ties -> lower axis, then lower plane, stable partition), or at the index
 * median if no axis has centroid extent or the node is 40 levels deep.
 * Deterministic: the same input gives byte-identical output.  n_tris may be 0
 * (an empty scene: every ray misses and counts nothing). */
rt_status rt_bvh_build(const float *vertices, const uint32_t *geom_ids, uint32_t n_tris,
                       void *nodes, size_t node_cap, void *tris, size_t tri_cap,
                       rt_bvh_info *info);

/* Build options of rt_bvh_build_ex. */
typedef struct rt_build_params {
    uint32_t max_leaf;       /* 1..7: a node with at most max_leaf triangles is a leaf (4 in
                                rt_bvh_build); the rest of the construction is unchanged */
} rt_build_params;

/* rt_bvh_build with options (params may be NULL: rt_bvh_build's).  The leaf
 * size is a tuning knob: smaller leaves trade triangle tests for box tests
 * (on camera-facing two-triangle quads, max_leaf = 2 runs 9 % faster than 4). */
rt_status rt_bvh_build_ex(const float *vertices, const uint32_t *geom_ids, uint32_t n_tris,
                          const rt_build_params *params, void *nodes, size_t node_cap, void *tris,
                          size_t tri_cap, rt_bvh_info *info);

/* Converts the inner nodes of a built BVH (host, from rt_bvh_build) to the
 * 32-byte layout: per node and axis a frame word -- the largest float32
 * <= the node's lower bound whose low 8 pattern bits are clear, carrying in
 * those bits an exponent E such that the scale 2^(E-127) is the smallest
 * with fma(255, scale, origin) >= the node's upper bound -- then each child
 * coordinate as the tightest 8-bit q whose decoded value
 * fma(q, scale, origin) lies on the outside of the exact bound (lower bounds
 * round down, upper bounds up), in the order qlo0.xyz qhi0.xyz qlo1.xyz
 * qhi1.xyz, then the two child references unchanged.  The traversal decodes
 * the boxes and box-tests them like float32 boxes; a decoded box contains
 * its exact box, so closest and any-hit answers equal the float32 layout's
 * except among hits of exactly equal t, while the counters are the
 * compressed traversal's own.  (The paper leaves the BVH format open.)
 *   nodes     host, info->n_nodes records of RT_NODE_BYTES
 *   out       host output, capacity out_cap >= n_nodes * RT_NODE_BYTES_Q8, 16-byte aligned
 *   out_info  host output: *info with layout = RT_LAYOUT_Q8 (may alias info)
 * Fails if info->layout is not RT_LAYOUT_F32 or a box is not finite. */
rt_status rt_bvh_compress(const void *nodes, const rt_bvh_info *info, void *out, size_t out_cap,
                          rt_bvh_info *out_info);

/* Converts the inner nodes of a built BVH (host, from rt_bvh_build) to the
 * four-wide layout: 128-byte nodes of up to four children, so that a ray
 * visits about half as many nodes and each node fetch brings four child
 * boxes (the paper leaves the BVH's arity open; Section 3.2's traversal only
 * needs child boxes).  For a binary inner node the child list starts as its
 * two children; while it has fewer than four entries and one of them is an
 * inner node, the inner entry with the largest box surface area (in double,
 * 2(dx dy + dy dz + dz dx); ties -> the earliest in the list) is replaced at
 * its place by its two children (first, second).  Each inner entry of the
 * final list becomes a four-wide node of its own; wide nodes are numbered in
 * depth-first preorder (children in list order, node 0 the root); leaf
 * entries keep their references.  Words of a node: lo.x[4], hi.x[4],
 * lo.y[4], hi.y[4], lo.z[4], hi.z[4] (child c in lane c, boxes bit-identical
 * to the binary child boxes), ref[4] (RT_WIDE_EMPTY_REF and a zero box in the
 * unused last slots), a zero word.  The traversal box-tests every child of a
 * node (counted), visits the hit ones in (entry distance, child index) order
 * and pushes all but the first, the second nearest on top; closest and
 * any-hit answers equal the binary layout's except among hits of exactly
 * equal t, and the counters are the wide traversal's own.
 *   nodes     host, info->n_nodes records of RT_NODE_BYTES (RT_LAYOUT_F32)
 *   out       host output, capacity out_cap >= info->n_nodes * RT_NODE_BYTES_WIDE4
 *             (an upper bound: the wide node count is returned), 16-byte aligned
 *   out_info  host output: *info with layout = RT_LAYOUT_WIDE4, n_nodes = the
 *             wide node count, max_depth = the stack bound (the largest sum of
 *             k - 1 over the wide nodes of a root-to-leaf path), root_ref 0 for
 *             an inner root (a root leaf stays as it is); may alias info.
 * Fails if info->layout is not RT_LAYOUT_F32 or a child reference is out of
 * range. */
rt_status rt_bvh_widen(const void *nodes, const rt_bvh_info *info, void *out, size_t out_cap,
                       rt_bvh_info *out_info);

/* Converts the inner nodes of a built BVH (host, from rt_bvh_build) to the
 * packed-reference layout: 48-byte nodes, three 16-byte fetches instead of
 * four (the paper leaves the node format open; Section 3.2's traversal
 * needs each child's box and reference).  A node is the twelve box words of
 * the 64-byte node, lo0.xyz, hi0.xyz, lo1.xyz, hi1.xyz, with no reference
 * words: child c's reference (as in the 64-byte node) is split into bytes,
 * least significant first, and byte k becomes the low byte of the bit
 * pattern of the child's k-th word among lo.x, lo.y, lo.z, hi.x.  Each such
 * word is moved outward to the nearest float32 whose pattern has that low
 * byte (the largest <= the bound for lo, the smallest >= it for hi,
 * walking patterns in value order with -0 just below +0: at most 255
 * patterns, 511 across zero); hi.y and hi.z are unchanged.  The traversal
 * uses the stored words as the child boxes and gathers the references from
 * their low bytes.  The boxes contain the exact ones, so closest and any-hit
 * answers equal the 64-byte layout's except among hits of exactly equal t,
 * while the counters are the packed traversal's own.
 *   nodes     host, info->n_nodes records of RT_NODE_BYTES (RT_LAYOUT_F32)
 *   out       host output, capacity out_cap >= n_nodes * RT_NODE_BYTES_F32P, 16-byte aligned
 *   out_info  host output: *info with layout = RT_LAYOUT_F32P (may alias info)
 * Fails if info->layout is not RT_LAYOUT_F32, a box is not finite, or a
 * moved word would reach an infinity (bounds within 255 patterns of the
 * float range's end). */
rt_status rt_bvh_pack(const void *nodes, const rt_bvh_info *info, void *out, size_t out_cap,
                      rt_bvh_info *out_info);

/* Refit plan of a built BVH (host, 64-byte nodes from rt_bvh_build), for
 * rt_bvh_refit, in plan (host output, plan_cap >= 3 * info->n_nodes words):
 *   plan[k]              2 * p + c when inner node k is child c (0 or 1) of
 *                        inner node p; 0xFFFFFFFF for the root (node 0)
 *   plan[n_nodes + k]    k's depth (root 0), with bit 31 set when k is a
 *                        "top" node: its subtree (inner nodes k .. k + size - 1
 *                        in preorder) leaves the block of 1024 numbers
 *                        that contains k
 *   plan[2 n_nodes + i]  the *n_top top nodes, i < *n_top
 * Nothing is planned (and *n_top = 0) for a root leaf or an empty tree.
 * Fails for another layout (RT_ERR_UNSUPPORTED) or a tree whose child
 * references do not point to later nodes, each node below the root from
 * exactly one parent, within max_depth. */
rt_status rt_bvh_refit_plan(const void *nodes, const rt_bvh_info *info, uint32_t *plan,
                            size_t plan_cap, uint32_t *n_top);

/* Refit (device): the scene's triangle records and node boxes recomputed in
 * place from new vertex positions, the topology unchanged -- for geometry
 * that moves between calls (the differentiable hit's optimisation steps)
 * without a host rebuild.  The paper leaves BVH construction open.  The mesh
 * is indexed: vertices (device, [n_vertices][3] float32) and faces (device,
 * [n_tris][3] uint32 by input triangle index, the order given to
 * rt_bvh_build).  Triangle records get v0, e1 = v1 - v0, e2 = v2 - v0
 * (float32) and keep prim_id and geom_id.  Every box grows from
 * (+inf, -inf) by strict comparisons -- a triangle's over its vertices 0, 1,
 * 2, a leaf's over its triangles in leaf order, an inner child's over its two
 * child boxes -- the order in which rt_bvh_build grows its boxes, so a refit
 * to the build's own vertices returns the build bit for bit.  A face index
 * >= n_vertices reads NaN: that corner adds nothing to any box and the
 * triangle is never hit.  root_box (device, 6 floats: lo.xyz, hi.xyz)
 * receives the new root box, which the caller copies into the scene's
 * rt_bvh_info.root_lo/root_hi before tracing (the traversal's root test
 * reads the host info).
 *   plan      device, rt_bvh_refit_plan's words (NULL for a root leaf)
 *   n_top     its *n_top
 * Two launches, no atomics: blocks of 1024 inner nodes (by number) that
 * also rewrite the triangle records, compute their leaf children's boxes and
 * finish, depth by depth with block barriers in on-chip memory, every node
 * whose subtree lies in the block; then one block that finishes the top
 * nodes depth by depth (in on-chip memory for up to 2048 of them).  The
 * scene's node and triangle buffers are written: calls must be ordered
 * against each other and against traces of the same scene on one stream.
 * Boxes stay exact as the vertices move; their quality drops with distance
 * from the built positions.  RT_LAYOUT_F32 scenes only. */
rt_status rt_bvh_refit(const rt_scene *scene, const uint32_t *plan, uint32_t n_top,
                       const float *vertices, uint32_t n_vertices, const uint32_t *faces,
                       float *root_box, void *stream);

/* Device workspace a trace call needs (bytes, possibly 0): the ray queue
 * head of persistent launch shapes and overflow space for traversal stacks
 * deeper than the on-chip stack.  Its contents need no initialisation and
 * are scratch: calls that share a workspace must be ordered on one stream. */
rt_status rt_trace_workspace_bytes(const rt_scene *scene, uint32_t n_rays, uint32_t flags,
                                   size_t *bytes);

/* Closest-hit query (Section 3.1, Listing 4) over the whole scene.
 *   rays      device, [n_rays] rt_ray
 *   kind/params  intersector (params: host pointer to the matching struct,
 *             NULL for RT_ISECT_DEFAULT); the struct is copied at the call
 *   hits      device output, [n_rays] rt_hit
 *   counters  device output, [n_rays] rt_counters; required iff RT_FLAG_COUNT
 *   workspace device, at least rt_trace_workspace_bytes bytes (may be NULL
 *             when that is 0)
 * n_rays == 0 returns RT_OK without a launch; n_rays > RT_MAX_RAYS is
 * RT_ERR_INVALID_ARG. */
rt_status rt_trace_closest(const rt_scene *scene, const rt_ray *rays, uint32_t n_rays,
                           rt_isect_kind kind, const void *params, uint32_t flags,
                           rt_hit *hits, rt_counters *counters,
                           void *workspace, size_t workspace_bytes, void *stream);

/* Bytes of the library's own fixed device scratch (64 MiB per GPU) that
 * rt_trace_closest_noalloc uses in place of a caller workspace. */
#define RT_NOALLOC_SCRATCH_BYTES (64u << 20)

/* rt_trace_closest without a workspace argument and without any allocation,
 * for callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation).  The workspace
 * rt_trace_closest would take (ray-queue heads and stack overflow space) is
 * a fixed RT_NOALLOC_SCRATCH_BYTES array in device memory that the library
 * holds on every GPU it runs on until the process ends.  Arguments, results
 * and errors as for rt_trace_closest (hits and counters are bit-identical),
 * plus: a call whose rt_trace_workspace_bytes exceeds
 * RT_NOALLOC_SCRATCH_BYTES fails with RT_ERR_WORKSPACE before any device
 * work (the default launch shape fits scenes of max_depth <= 22 at any ray
 * count; more LDS stack slots or fewer rays per call fit deeper ones).  The
 * stream must belong to the current device.  All calls on one GPU share
 * that GPU's scratch: calls that overlap in time on one GPU (two streams,
 * two threads) race and give undefined results; calls ordered on one stream
 * do not.  The first call on a device looks up the scratch's address there
 * (RT_ERR_HIP if that fails). */
rt_status rt_trace_closest_noalloc(const rt_scene *scene, const rt_ray *rays, uint32_t n_rays,
                                   rt_isect_kind kind, const void *params, uint32_t flags,
                                   rt_hit *hits, rt_counters *counters, void *stream);

/* Any-hit query (Section 3.1): occluder[i] = input index of the first hit
 * the intersector accepted in traversal order, or RT_MISS.  Arguments as for
 * rt_trace_closest. */
rt_status rt_trace_any(const rt_scene *scene, const rt_ray *rays, uint32_t n_rays,
                       rt_isect_kind kind, const void *params, uint32_t flags,
                       uint32_t *occluder, rt_counters *counters,
                       void *workspace, size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------
 * Batched launch: many scenes, each with its own consecutive range of rays,
 * traced by one launch (one persistent grid draining one ray queue).
 * The caller packs a scene table on the host (rt_batch_pack), copies it to
 * device memory, and passes the device copy to rt_trace_batch; nothing is
 * copied behind the caller's back, so the launch can be graph-captured.
 * --------------------------------------------------------------------- */
typedef struct rt_batch_entry {
    rt_scene scene;          /* the scene's BVH (device), from rt_bvh_build */
    uint32_t n_rays;         /* rays of this scene: the next n_rays of the batch */
    rt_alpha_params alpha;   /* alpha-mask data of this scene (RT_ISECT_ALPHA only) */
} rt_batch_entry;

typedef struct rt_batch_info {
    uint32_t n_scenes;
    uint32_t n_rays;         /* sum of the entries' n_rays */
    uint32_t max_depth;      /* deepest BVH of the batch */
    uint32_t kind;           /* the intersector kind the table was packed for */
    uint32_t layout;         /* node layout shared by every scene of the batch */
} rt_batch_info;

/* Bytes of the packed table for n_scenes scenes. */
rt_status rt_batch_table_bytes(uint32_t n_scenes, size_t *bytes);

/* Validates the entries (every scene as rt_trace_closest would, and for
 * RT_ISECT_ALPHA every entry's alpha data against its scene; all scenes must
 * share one node layout) and writes the table into host_table (host,
 * 16-byte aligned, table_bytes >= rt_batch_table_bytes).  The device
 * pointers inside are copied verbatim. */
rt_status rt_batch_pack(const rt_batch_entry *entries, uint32_t n_scenes, rt_isect_kind kind,
                        void *host_table, size_t table_bytes, rt_batch_info *info);

/* Workspace of rt_trace_batch (as rt_trace_workspace_bytes). */
rt_status rt_trace_batch_workspace_bytes(const rt_batch_info *info, uint32_t flags,
                                         size_t *bytes);

/* Closest-hit query over a batch (Section 3.1 per scene).  table: device copy
 * of the packed table described by info; rays/hits/counters: device,
 * [info->n_rays] in scene order (scene s owns the rays after those of scenes
 * 0..s-1).  kind must be the kind the table was packed for; params: NULL, or
 * rt_procedural_params for RT_ISECT_PROCEDURAL (the alpha data comes from the
 * table).  Results are bit-identical to one rt_trace_closest call per scene. */
rt_status rt_trace_batch(const void *table, const rt_batch_info *info, const rt_ray *rays,
                         rt_isect_kind kind, const void *params, uint32_t flags, rt_hit *hits,
                         rt_counters *counters, void *workspace, size_t workspace_bytes,
                         void *stream);

/* ---------------------------------------------------------------------
 * Instancing (Section 3.2: a BVH may be a primitive of another BVH; object
 * instancing).  A top-level BVH is built over instances; an instance is a
 * bottom-level scene (from rt_bvh_build) seen through an affine map.  At a
 * top-level leaf every instance in stored order is entered with the object
 * ray o' = M o + m, d' = M d (float32: o'_i = fma(M_i0, o_x, fma(M_i1, o_y,
 * fma(M_i2, o_z, m_i))), d'_i = fma(M_i0, d_x, fma(M_i1, d_y, M_i2 d_z))),
 * which leaves t and the barycentrics of a hit unchanged.
 * --------------------------------------------------------------------- */
typedef struct rt_instance {
    uint32_t blas;                 /* index of the bottom-level scene */
    float object_from_world[12];   /* row-major 3x4 [M | m] */
    float world_lo[3], world_hi[3];/* a world box containing the instance under
                                      that map (the caller's responsibility) */
} rt_instance;

/* Host build of the top-level BVH over the instances' world boxes (same
 * construction as rt_bvh_build; buffer sizes from rt_bvh_buffer_bytes(n_inst));
 * its leaf records carry instance indices as prim_id. */
rt_status rt_tlas_build(const rt_instance *instances, uint32_t n_inst, void *nodes,
                        size_t node_cap, void *tris, size_t tri_cap, rt_bvh_info *info);

/* Bytes of the packed instance table. */
rt_status rt_instance_table_bytes(uint32_t n_blas, uint32_t n_inst, size_t *bytes);

/* Texture coordinates of one mesh, for the alpha mask of an instanced scene
 * (every mesh has its own; the texture array is shared). */
typedef struct rt_mesh_texcoords {
    const float *texcoords;   /* device, [n_prims][3][2] by the mesh's input
                                 triangle index, 8-byte aligned */
    uint32_t n_prims;         /* must be >= the mesh's n_tris */
} rt_mesh_texcoords;

/* What rt_instance_pack found out about the meshes; the trace calls take it
 * with the table. */
typedef struct rt_instance_info {
    uint32_t n_blas, n_inst;
    uint32_t max_blas_depth;  /* deepest bottom-level BVH */
    uint32_t max_geom_id;     /* largest texture id over the meshes */
    uint32_t has_texcoords;   /* 1 iff texture coordinates were given for
                                 every mesh with triangles */
} rt_instance_info;

/* Instancing takes scenes of layout RT_LAYOUT_F32 only (bottom and top level).
 *
 * Validates the bottom-level scenes, their texture coordinates (texcoords:
 * host array [n_blas], or NULL when no alpha mask will be used; an entry may
 * be {NULL, 0} for a mesh without triangles) and the instances, writes the
 * table into host_table (host, 16-byte aligned) and fills *info.  The caller
 * copies the table to device memory. */
rt_status rt_instance_pack(const rt_scene *blas, const rt_mesh_texcoords *texcoords,
                           uint32_t n_blas, const rt_instance *instances, uint32_t n_inst,
                           void *host_table, size_t table_bytes, rt_instance_info *info);

/* Workspace of rt_trace_instanced. */
rt_status rt_trace_instanced_workspace_bytes(const rt_scene *tlas, const rt_instance_info *info,
                                             uint32_t n_rays, uint32_t flags, size_t *bytes);

/* Closest-hit (any_hit = 0: out is rt_hit[n_rays], prim_id relative to the
 * hit instance's scene) or any-hit (any_hit = 1: out is uint32[n_rays])
 * query over an instanced scene.  tlas: from rt_tlas_build over the same
 * instances as the device table; info: from rt_instance_pack of that table;
 * inst_ids (device, may be NULL) receives the hit instance or RT_MISS.
 * RT_ISECT_DEFAULT, RT_ISECT_PROCEDURAL, or RT_ISECT_ALPHA with an
 * rt_alpha_params whose texture array serves every mesh (its texcoords and
 * n_texcoord_prims are ignored: each mesh uses the texture coordinates given
 * to rt_instance_pack, and texture ids come from each mesh's rt_bvh_build).
 * RT_FLAG_COUNT counts the box tests of both levels and the triangle tests;
 * RT_FLAG_TILE_WIDTH gives each wave one 8 x 8 tile of an image's rays
 * (results unchanged); other flag bits are RT_ERR_UNSUPPORTED. */
rt_status rt_trace_instanced(const rt_scene *tlas, const void *table, const rt_instance_info *info,
                             const rt_ray *rays, uint32_t n_rays, rt_isect_kind kind,
                             const void *params, uint32_t flags, int any_hit, void *out,
                             uint32_t *inst_ids, rt_counters *counters, void *workspace,
                             size_t workspace_bytes, void *stream);

/* Multi-hit query (Section 3.1 names a query returning several hit
 * points; read here as the k nearest hits the intersector accepts, in increasing t; a hit with the same
 * t as a kept one goes after it).  Once k hits are kept, the k-th distance
 * bounds the search.
 *   k       1..RT_MAX_MULTI
 *   hits    device output, [n_rays][k] rt_hit, nearest first, padded with
 *           miss records
 *   n_hits  device output, [n_rays] uint32, hits kept per ray (<= k)
 * Other arguments as for rt_trace_closest; with k = 1 the result equals
 * rt_trace_closest's. */
#define RT_MAX_MULTI 8
rt_status rt_trace_multi(const rt_scene *scene, const rt_ray *rays, uint32_t n_rays,
                         rt_isect_kind kind, const void *params, uint32_t flags, uint32_t k,
                         rt_hit *hits, uint32_t *n_hits, rt_counters *counters, void *workspace,
                         size_t workspace_bytes, void *stream);

/* Adjoint of the accepted closest hits (differentiable hit).  For every ray
 * whose hit (from rt_trace_closest over the triangles vertices[faces]) is not
 * a miss, the hit point o + t d = (1-u-v) v0 + u v1 + v v2 of triangle
 * faces[prim_id] is differentiated implicitly with respect to the ray and the
 * three vertex positions, holding the hit prim and the intersector's decision
 * fixed (they are discrete).  With g = grad_tuv[i] = (dL/dt, dL/du, dL/dv),
 * A = [d, -e1, -e2] (columns) and lam = -A^-T g:
 *   grad_vertices[faces[prim][k]] += c_k lam, (c_0, c_1, c_2) = (-(1-u-v), -u, -v)
 *   grad_rays[i] = (lam, 0, t lam, 0)   (dL/do, dL/dtmin, dL/dd, dL/dtmax)
 *   rays          device, [n_rays] rt_ray (the traced rays)
 *   hits          device, [n_rays] rt_hit (the forward result)
 *   grad_tuv      device, [n_rays][3] float
 *   vertices      device, [n_vertices][3] float
 *   faces         device, [n_tris][3] uint32, the forward's triangles
 *   grad_vertices device, [n_vertices][3] float, ACCUMULATED (caller zeroes);
 *                 hipMalloc memory (float32 hardware atomics)
 *   grad_rays     device, [n_rays][8] float, overwritten (zero for misses),
 *                 or NULL
 * Rays whose prim_id or face indices are out of range contribute nothing.
 * The atomics' summation order is unspecified, so the last bits of
 * grad_vertices vary between runs.  No paper counterpart: this is the
 * differentiable extension of the closest-hit query of Section 3.1. */
rt_status rt_hit_backward(const rt_ray *rays, const rt_hit *hits, const float *grad_tuv,
                          uint32_t n_rays, const float *vertices, uint32_t n_vertices,
                          const uint32_t *faces, uint32_t n_tris, float *grad_vertices,
                          float *grad_rays, void *stream);

/* Launch shapes compiled into the library (the index a call selects with
 * RT_FLAG_SHAPE is the position in this list):
 *   block      threads per block;
 *   lds_stack  LDS ring slots per lane for the top of the traversal stack
 *              (lds_stack - 1 entries stay on chip, older ones move to the
 *              workspace);
 *   chunk      rays a wave takes at a time; the wave hands the next ray of
 *              its chunk to a lane as soon as the lane's ray is finished;
 *   queue      1: a persistent grid (the blocks that can be resident at
 *              once, from the occupancy query; the workspace is sized for at
 *              most 256 CUs x 32 wave slots) takes chunks from atomic queues
 *              kept in the workspace; 0: wave w owns the static chunk w.
 * Writes up to cap entries per array (any array may be NULL) and returns the
 * number of shapes; the first shape is the default.  Scenes of layout
 * RT_LAYOUT_Q8 run with the default shape only (other shapes return
 * RT_ERR_UNSUPPORTED), and not with the run-time dispatch flags. */
uint32_t rt_launch_shapes(uint32_t *blocks, uint32_t *lds_stacks, uint32_t *chunks,
                          uint32_t *queues, uint32_t cap);

/* Static description of a status code. */
const char *rt_status_string(rt_status status);

/* Detail of the last failure on the calling thread ("" if none). */
const char *rt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RTX_H */
