/*
 * rt_oracle.c -- CPU oracle for custom-intersector ray traversal.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or table with the GPU library.
 *
 * Two oracles, both plain and slow on purpose:
 *
 * A. orc_brute  -- the plain definition of the visibility queries
 *    (Section 3.1: closest-hit returns the nearest accepted hit, any-hit the
 *    first one encountered).  Section 3.2 notes that a query may run over a
 *    linear primitive list with no BVH at all and must give the same answer,
 *    so oracle A tests every ray against every triangle in float64.  The
 *    ray/triangle test is the plane-then-area-ratio formulation (not the
 *    one the GPU uses), and the intersector (Section 4: alpha mask, procedural
 *    mask) is evaluated in float64 on the float64 barycentrics.
 *    It also reports, per ray, the second-nearest accepted distance and the
 *    flags of the exception set (near-ties, near-edge hits, near filter
 *    decisions) together with an a-priori float32 forward-error bound.
 *
 * B. orc_build + orc_traverse -- the BVH heat-map counts of Section 4 (the
 *    counting intersector increments one counter per ray/box test and one per
 *    ray/triangle test) depend on the BVH and on the traversal order, so they
 *    have no order-free definition.  Oracle B builds its own BVH (binned SAH,
 *    the reading documented with the build) and walks it with the while-while
 *    scheme of Algorithm 1 in float32, the precision of the paper's
 *    basic_triangle<3, float>; box tests are intercepted for counting, and
 *    triangle tests are followed by the intersector's accept decision, whose
 *    result is AND-ed into the hit (Listing 3 / Listing 5 semantics).
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared -pthread -lm.
 * -ffp-contract=off matters: every fused multiply-add below is an explicit
 * fma()/fmaf() call and nothing else may be contracted.
 */
#include <float.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MISS 0xFFFFFFFFu
#define ORC_MAX_MULTI 8

enum { ORC_DEFAULT = 0, ORC_ALPHA = 1, ORC_PROCEDURAL = 2 };

/* Exception-set flag bits reported by oracle A. */
enum {
    ORC_E_NEAR_TIE = 1u,      /* two nearest accepted t within 1e-6 relative */
    ORC_E_NEAR_EDGE = 2u,     /* a relevant candidate within delta of an edge */
    ORC_E_NEAR_FILTER = 4u,   /* a relevant accept decision within delta of its boundary */
};

typedef struct {
    const float *texcoords;   /* [n_prims][3][2], by input triangle index */
    const uint32_t *textures; /* [n_tex][height][width] RGBA8, alpha in the high byte */
    uint32_t n_tex, width, height;
    uint32_t alpha_min;       /* accept iff alpha byte >= alpha_min */
    uint32_t checker_n;       /* procedural: accept iff floor(n u)+floor(n v) even */
} orc_isect;

/* ======================================================================
 * Oracle A: float64 brute force
 * ====================================================================== */

typedef struct { double x, y, z; } d3;

static d3 d3_sub(d3 a, d3 b) { d3 r = {a.x - b.x, a.y - b.y, a.z - b.z}; return r; }
static d3 d3_add(d3 a, d3 b) { d3 r = {a.x + b.x, a.y + b.y, a.z + b.z}; return r; }
static d3 d3_scale(d3 a, double s) { d3 r = {a.x * s, a.y * s, a.z * s}; return r; }
static double d3_dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static d3 d3_cross(d3 a, d3 b)
{
    d3 r = {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
    return r;
}
static double d3_norm(d3 a) { return sqrt(d3_dot(a, a)); }
static d3 d3_load(const float *p) { d3 r = {p[0], p[1], p[2]}; return r; }

/* Distance of x to the nearest integer. */
static double frac_dist(double x) { return fabs(x - floor(x + 0.5)); }

/* Alpha-mask decision (Section 4, Listing 5) in float64: interpolate the
 * three texture coordinates with weights (1-u-v, u, v), take the nearest texel
 * (clamp to edge) of texture geom_id and compare its alpha byte. */
static int alpha_texel_ok(const orc_isect *is, uint32_t geom, double xs, double ys)
{
    double xf = floor(xs), yf = floor(ys);
    if (xf < 0) xf = 0;
    if (xf > is->width - 1.0) xf = is->width - 1.0;
    if (yf < 0) yf = 0;
    if (yf > is->height - 1.0) yf = is->height - 1.0;
    uint32_t texel = is->textures[((size_t)geom * is->height + (size_t)yf) * is->width + (size_t)xf];
    return (texel >> 24) >= is->alpha_min;
}

static void alpha_lookup64(const orc_isect *is, uint32_t prim, double u, double v,
                           double *xs, double *ys)
{
    const float *tc = is->texcoords + (size_t)prim * 6;
    double w0 = 1.0 - u - v;
    double s = w0 * tc[0] + u * tc[2] + v * tc[4];
    double t = w0 * tc[1] + u * tc[3] + v * tc[5];
    *xs = s * is->width;
    *ys = t * is->height;
}

static int alpha_accept64(const orc_isect *is, uint32_t prim, uint32_t geom, double u, double v)
{
    double xs, ys;
    alpha_lookup64(is, prim, u, v, &xs, &ys);
    return alpha_texel_ok(is, geom, xs, ys);
}

/* 1 iff a lookup displaced by at most `reach` texels on each axis could land
 * on a texel whose accept decision differs from the undisplaced one. */
static int alpha_decision_fragile(const orc_isect *is, uint32_t prim, uint32_t geom,
                                  double u, double v, double reach)
{
    double xs, ys;
    alpha_lookup64(is, prim, u, v, &xs, &ys);
    int ok = alpha_texel_ok(is, geom, xs, ys);
    if (!(reach < (double)is->width && reach < (double)is->height)) return 1;
    double x0 = floor(xs - reach), x1 = floor(xs + reach);
    double y0 = floor(ys - reach), y1 = floor(ys + reach);
    for (double y = y0; y <= y1; y += 1.0)
        for (double x = x0; x <= x1; x += 1.0)
            if (alpha_texel_ok(is, geom, x + 0.5, y + 0.5) != ok) return 1;
    return 0;
}

/* Procedural checker in float64; *margin is the distance of n*u or n*v to an
 * integer. */
static int checker_accept64(const orc_isect *is, double u, double v, double *margin)
{
    double n = (double)is->checker_n;
    double a = floor(n * u), b = floor(n * v);
    double mu = frac_dist(n * u), mv = frac_dist(n * v);
    *margin = mu < mv ? mu : mv;
    long long k = (long long)a + (long long)b;
    return (k % 2) == 0;
}

typedef struct {
    const float *verts;       /* [n_tris][3][3] */
    const uint32_t *geom;     /* [n_tris] or NULL */
    uint32_t n_tris;
    const float *rays;        /* [n_rays][8] */
    const int64_t *ray_index; /* optional subset of rays (NULL = all) */
    uint32_t n_rays;
    int kind;
    orc_isect is;
    int any_hit;
    /* outputs, indexed like the (sub)set */
    double *t, *u, *v, *t2, *bound_uv, *bound_t;
    uint32_t *prim;
    uint8_t *flags;
    /* work distribution */
    uint32_t next;
    pthread_mutex_t lock;
} brute_job;

/* One candidate evaluation in float64.  Returns 1 iff the ray meets the
 * triangle's plane (d.n != 0); then t, u, v, the edge margin
 * min(u, v, 1-u-v) and the float32 error bounds are filled in. */
static int plane_hit64(d3 o, d3 d, const float *tri, double *t, double *u, double *v,
                       double *margin, double *b_uv, double *b_t)
{
    d3 v0 = d3_load(tri), v1 = d3_load(tri + 3), v2 = d3_load(tri + 6);
    d3 e1 = d3_sub(v1, v0), e2 = d3_sub(v2, v0);
    d3 n = d3_cross(e1, e2);
    double dn = d3_dot(d, n);
    if (dn == 0.0) return 0;
    double tt = d3_dot(d3_sub(v0, o), n) / dn;
    d3 p = d3_add(o, d3_scale(d, tt));
    d3 w = d3_sub(p, v0);
    double nn = d3_dot(n, n);
    double uu = d3_dot(d3_cross(w, e2), n) / nn;
    double vv = d3_dot(d3_cross(e1, w), n) / nn;
    *t = tt; *u = uu; *v = vv;
    double m = uu < vv ? uu : vv;
    double w0 = 1.0 - uu - vv;
    *margin = m < w0 ? m : w0;
    /* A-priori forward-error bound of a float32 Moller-Trumbore evaluation
     * from the same float32 inputs (unit roundoff eps = 2^-24).  Term by term:
     * s = o - v0, e1, e2 are each rounded once (eps relative); p = d x e2 and
     * q = s x e1 carry under 5 eps of their operand norms; each three-term
     * fma dot product adds 3 eps; the reciprocal and the final products add
     * 2 eps.  Summed, |du|, |dv| <= 8 eps |d| (|s|(|e1|+|e2|) + |e1||e2|)/|det|
     * + 2 eps and |dt| <= 9 eps |e1||e2| (|s| + |t||d|)/|det| + 2 eps |t|,
     * with |det| = |d.(e1 x e2)|.  The constants are rounded up (10 and 4) to
     * absorb the difference between the float32 and exact det. */
    const double eps = 0x1p-24;
    double nd = d3_norm(d), ne1 = d3_norm(e1), ne2 = d3_norm(e2);
    double ns = d3_norm(d3_sub(o, v0));
    double adet = fabs(dn);
    *b_uv = 10.0 * eps * nd * (ns * (ne1 + ne2) + ne1 * ne2) / adet + 4.0 * eps;
    *b_t = 10.0 * eps * ne1 * ne2 * (ns + fabs(tt) * nd) / adet + 4.0 * eps * fabs(tt);
    return 1;
}

static void brute_one(brute_job *job, uint32_t slot)
{
    int64_t ri = job->ray_index ? job->ray_index[slot] : (int64_t)slot;
    const float *r = job->rays + (size_t)ri * 8;
    d3 o = {r[0], r[1], r[2]}, d = {r[4], r[5], r[6]};
    double tmin = r[3], tmax = r[7];
    double t1 = INFINITY, t2 = INFINITY, u1 = 0, v1 = 0, bu1 = 0, bt1 = 0;
    uint32_t p1 = ORC_MISS;

    /* Pass 1: nearest and second-nearest accepted hit (ties -> lowest index).
     * Any-hit keeps the same nearest record: its hit/miss answer is the
     * existence of an accepted hit, and the nearest is one such hit. */
    for (uint32_t k = 0; k < job->n_tris; ++k) {
        double t, u, v, m, bu, bt;
        if (!plane_hit64(o, d, job->verts + (size_t)k * 9, &t, &u, &v, &m, &bu, &bt)) continue;
        if (!(m >= 0.0) || !(t > tmin) || !(t < tmax)) continue;
        int acc = 1;
        double fm;
        if (job->kind == ORC_ALPHA)
            acc = alpha_accept64(&job->is, k, job->geom ? job->geom[k] : 0, u, v);
        else if (job->kind == ORC_PROCEDURAL)
            acc = checker_accept64(&job->is, u, v, &fm);
        if (!acc) continue;
        if (t < t1) {
            t2 = t1;
            t1 = t; u1 = u; v1 = v; p1 = k; bu1 = bu; bt1 = bt;
        } else if (t < t2) {
            t2 = t;
        }
    }

    /* Pass 2: exception flags.  Candidates that matter are those whose
     * plane distance lies inside (tmin, tmax) and no farther than the nearest
     * accepted hit (plus 1e-6 relative); for a miss, every such candidate. */
    uint8_t fl = 0;
    if (p1 != ORC_MISS && t2 - t1 < 1e-6 * fabs(t1)) fl |= ORC_E_NEAR_TIE;
    double reach = (p1 != ORC_MISS) ? t1 + 1e-6 * fabs(t1) + bt1 : tmax;
    for (uint32_t k = 0; k < job->n_tris; ++k) {
        double t, u, v, m, bu, bt;
        if (!plane_hit64(o, d, job->verts + (size_t)k * 9, &t, &u, &v, &m, &bu, &bt)) continue;
        if (!(t > tmin - bt) || !(t < tmax + bt) || !(t <= reach + bt)) continue;
        double delta = bu > 1e-6 ? bu : 1e-6;
        if (fabs(m) < delta) fl |= ORC_E_NEAR_EDGE;
        if (m > -delta && job->kind != ORC_DEFAULT) {
            double fm = 1.0;
            if (job->kind == ORC_ALPHA) {
                /* s = w0 tc0 + u tc1 + v tc2 with texture coordinates in
                 * [0, 1] moves by at most 2 delta (+ float32 rounding), i.e.
                 * 2 delta W texels; the decision is fragile only if a texel
                 * within that reach decides differently. */
                double wh = job->is.width > job->is.height ? job->is.width : job->is.height;
                double reach = (2.0 * delta + 0x1p-20) * wh;
                if (alpha_decision_fragile(&job->is, k, job->geom ? job->geom[k] : 0, u, v, reach))
                    fl |= ORC_E_NEAR_FILTER;
            } else {
                checker_accept64(&job->is, u, v, &fm);
                if (fm < 2.0 * delta * job->is.checker_n) fl |= ORC_E_NEAR_FILTER;
            }
        }
        /* distance ties between distinct relevant candidates within the
         * float32 distance error also make the winner ambiguous */
        if (p1 != ORC_MISS && k != p1 && m > -delta && fabs(t - t1) <= bt + bt1)
            fl |= ORC_E_NEAR_TIE;
    }

    job->t[slot] = t1;
    job->u[slot] = u1;
    job->v[slot] = v1;
    job->t2[slot] = t2;
    job->prim[slot] = p1;
    job->flags[slot] = fl;
    job->bound_uv[slot] = bu1;
    job->bound_t[slot] = bt1;
}

static void *brute_worker(void *arg)
{
    brute_job *job = (brute_job *)arg;
    for (;;) {
        pthread_mutex_lock(&job->lock);
        uint32_t b = job->next;
        job->next = b + 64 < job->n_rays ? b + 64 : job->n_rays;
        uint32_t e = job->next;
        pthread_mutex_unlock(&job->lock);
        if (b >= e) break;
        for (uint32_t s = b; s < e; ++s) brute_one(job, s);
    }
    return NULL;
}

static void run_threads(void *(*fn)(void *), void *job, int n_threads)
{
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    pthread_t th[256];
    int started = 0;
    for (int i = 1; i < n_threads; ++i)
        if (pthread_create(&th[started], NULL, fn, job) == 0) ++started;
    fn(job);
    for (int i = 0; i < started; ++i) pthread_join(th[i], NULL);
}

/* Oracle A entry point.  ray_index may be NULL (all n_rays rays) or list the
 * n_rays ray indices to evaluate; outputs are indexed by position in that
 * list.  Misses: prim = ORC_MISS, t = +inf. */
int orc_brute(const float *verts, const uint32_t *geom_ids, uint32_t n_tris,
              const float *rays, const int64_t *ray_index, uint32_t n_rays,
              int kind, const orc_isect *is, int any_hit,
              double *t, uint32_t *prim, double *u, double *v, double *t2,
              uint8_t *flags, double *bound_uv, double *bound_t, int n_threads)
{
    if (kind < ORC_DEFAULT || kind > ORC_PROCEDURAL) return -1;
    brute_job job;
    memset(&job, 0, sizeof job);
    job.verts = verts; job.geom = geom_ids; job.n_tris = n_tris;
    job.rays = rays; job.ray_index = ray_index; job.n_rays = n_rays;
    job.kind = kind; job.any_hit = any_hit;
    if (is) job.is = *is;
    job.t = t; job.u = u; job.v = v; job.t2 = t2; job.prim = prim; job.flags = flags;
    job.bound_uv = bound_uv; job.bound_t = bound_t;
    pthread_mutex_init(&job.lock, NULL);
    run_threads(brute_worker, &job, n_threads);
    pthread_mutex_destroy(&job.lock);
    return 0;
}

/* ======================================================================
 * Oracle B part 1: BVH construction (binned SAH)
 *
 * The paper uses a BVH without describing its construction.  Reading used
 * here (and by the product builder, which is a separate implementation):
 *   - triangle box = exact float min/max of its vertices; centroid (float64)
 *     = 0.5 * (lo + hi);
 *   - a node with at most max_leaf triangles is a leaf (max_leaf in 1..7,
 *     4 by default);
 *   - otherwise, per axis with non-zero centroid extent, 32 equal-width bins
 *     over the centroid range, bin = min(31, (int)((c - cmin) * (32 / ext)));
 *     every plane between bins is a candidate with cost
 *     area(L) * |L| + area(R) * |R| (area = box surface in float64); the
 *     strictly smallest cost wins, ties keep the lower axis, then the lower
 *     plane; the node's triangles are stably partitioned;
 *   - when no axis has extent (all centroids equal), or the node sits at
 *     depth >= 40, the range is split at index count/2 in its current order;
 *   - nodes are numbered in depth-first preorder, left child first; each
 *     leaf owns a contiguous range of the final triangle order.
 * ====================================================================== */

typedef struct {
    float lo[3], hi[3];
    uint32_t left, right;  /* children (inner nodes) */
    uint32_t first, count; /* triangle range (leaves: count > 0) */
    uint32_t depth;
} orc_node;

typedef struct {
    const float *tri_lo, *tri_hi; /* [n][3] float boxes */
    const double *cen;            /* [n][3] centroids */
    uint32_t *perm, *tmp;
    orc_node *nodes;
    uint32_t n_nodes, cap;
    uint32_t max_depth;
    uint32_t max_leaf;
} build_ctx;

static double box_area(const float lo[3], const float hi[3])
{
    double dx = (double)hi[0] - (double)lo[0];
    double dy = (double)hi[1] - (double)lo[1];
    double dz = (double)hi[2] - (double)lo[2];
    return 2.0 * (dx * dy + dy * dz + dz * dx);
}

static void box_empty(float lo[3], float hi[3])
{
    for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
}

static void box_grow(float lo[3], float hi[3], const float *blo, const float *bhi)
{
    for (int a = 0; a < 3; ++a) {
        if (blo[a] < lo[a]) lo[a] = blo[a];
        if (bhi[a] > hi[a]) hi[a] = bhi[a];
    }
}

static int bin_of(double c, double cmin, double scale)
{
    int b = (int)((c - cmin) * scale);
    if (b > 31) b = 31;
    if (b < 0) b = 0;
    return b;
}

static uint32_t build_rec(build_ctx *ctx, uint32_t first, uint32_t count, uint32_t depth)
{
    uint32_t id = ctx->n_nodes++;
    orc_node *nd = &ctx->nodes[id];
    memset(nd, 0, sizeof *nd);
    nd->depth = depth;
    if (depth > ctx->max_depth) ctx->max_depth = depth;
    box_empty(nd->lo, nd->hi);
    for (uint32_t i = first; i < first + count; ++i) {
        uint32_t k = ctx->perm[i];
        box_grow(nd->lo, nd->hi, ctx->tri_lo + 3 * (size_t)k, ctx->tri_hi + 3 * (size_t)k);
    }
    if (count <= ctx->max_leaf) {
        nd->first = first;
        nd->count = count;
        return id;
    }

    double cmin[3] = {INFINITY, INFINITY, INFINITY}, cmax[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t i = first; i < first + count; ++i) {
        const double *c = ctx->cen + 3 * (size_t)ctx->perm[i];
        for (int a = 0; a < 3; ++a) {
            if (c[a] < cmin[a]) cmin[a] = c[a];
            if (c[a] > cmax[a]) cmax[a] = c[a];
        }
    }

    int best_axis = -1, best_plane = 0;
    double best_cost = INFINITY;
    if (depth < 40) {
        for (int a = 0; a < 3; ++a) {
            double ext = cmax[a] - cmin[a];
            if (!(ext > 0.0)) continue;
            double scale = 32.0 / ext;
            float blo[32][3], bhi[32][3];
            uint32_t bn[32];
            for (int b = 0; b < 32; ++b) { box_empty(blo[b], bhi[b]); bn[b] = 0; }
            for (uint32_t i = first; i < first + count; ++i) {
                uint32_t k = ctx->perm[i];
                int b = bin_of(ctx->cen[3 * (size_t)k + a], cmin[a], scale);
                bn[b]++;
                box_grow(blo[b], bhi[b], ctx->tri_lo + 3 * (size_t)k, ctx->tri_hi + 3 * (size_t)k);
            }
            /* candidate plane s: bins [0, s) left, [s, 32) right */
            for (int s = 1; s < 32; ++s) {
                float llo[3], lhi[3], rlo[3], rhi[3];
                uint32_t nl = 0, nr = 0;
                box_empty(llo, lhi);
                box_empty(rlo, rhi);
                for (int b = 0; b < s; ++b) { nl += bn[b]; if (bn[b]) box_grow(llo, lhi, blo[b], bhi[b]); }
                for (int b = s; b < 32; ++b) { nr += bn[b]; if (bn[b]) box_grow(rlo, rhi, blo[b], bhi[b]); }
                if (nl == 0 || nr == 0) continue;
                double cost = box_area(llo, lhi) * (double)nl + box_area(rlo, rhi) * (double)nr;
                if (cost < best_cost) { best_cost = cost; best_axis = a; best_plane = s; }
            }
        }
    }

    uint32_t nl;
    if (best_axis >= 0) {
        double scale = 32.0 / (cmax[best_axis] - cmin[best_axis]);
        uint32_t w = first, wr = 0;
        for (uint32_t i = first; i < first + count; ++i) {
            uint32_t k = ctx->perm[i];
            if (bin_of(ctx->cen[3 * (size_t)k + best_axis], cmin[best_axis], scale) < best_plane)
                ctx->perm[w++] = k;
            else
                ctx->tmp[wr++] = k;
        }
        nl = w - first;
        memcpy(ctx->perm + w, ctx->tmp, wr * sizeof(uint32_t));
    } else {
        nl = count / 2;
    }
    uint32_t l = build_rec(ctx, first, nl, depth + 1);
    uint32_t r = build_rec(ctx, first + nl, count - nl, depth + 1);
    nd = &ctx->nodes[id]; /* nodes[] does not move (preallocated) */
    nd->left = l;
    nd->right = r;
    return id;
}

/* Builds the oracle's BVH.  nodes must hold 2*n_tris (at least 1) entries.
 * Outputs: node array (preorder, node 0 = root), perm (leaf order -> input
 * triangle index), node count and maximum node depth. */
int orc_build_leaf(const float *verts, uint32_t n_tris, uint32_t max_leaf, orc_node *nodes,
                   uint32_t *perm, uint32_t *n_nodes_out, uint32_t *max_depth_out);

int orc_build(const float *verts, uint32_t n_tris, orc_node *nodes, uint32_t *perm,
              uint32_t *n_nodes_out, uint32_t *max_depth_out)
{
    return orc_build_leaf(verts, n_tris, 4, nodes, perm, n_nodes_out, max_depth_out);
}

/* The same build with leaves of at most max_leaf (1..7) triangles. */
int orc_build_leaf(const float *verts, uint32_t n_tris, uint32_t max_leaf, orc_node *nodes,
                   uint32_t *perm, uint32_t *n_nodes_out, uint32_t *max_depth_out)
{
    if (max_leaf < 1 || max_leaf > 7) return -2;
    if (n_tris == 0) {
        memset(&nodes[0], 0, sizeof nodes[0]);
        box_empty(nodes[0].lo, nodes[0].hi);
        *n_nodes_out = 1;
        *max_depth_out = 0;
        return 0;
    }
    float *tlo = malloc(sizeof(float) * 3 * n_tris);
    float *thi = malloc(sizeof(float) * 3 * n_tris);
    double *cen = malloc(sizeof(double) * 3 * n_tris);
    uint32_t *tmp = malloc(sizeof(uint32_t) * n_tris);
    if (!tlo || !thi || !cen || !tmp) { free(tlo); free(thi); free(cen); free(tmp); return -1; }
    for (uint32_t k = 0; k < n_tris; ++k) {
        const float *t = verts + 9 * (size_t)k;
        for (int a = 0; a < 3; ++a) {
            float lo = t[a], hi = t[a];
            if (t[3 + a] < lo) lo = t[3 + a];
            if (t[6 + a] < lo) lo = t[6 + a];
            if (t[3 + a] > hi) hi = t[3 + a];
            if (t[6 + a] > hi) hi = t[6 + a];
            tlo[3 * (size_t)k + a] = lo;
            thi[3 * (size_t)k + a] = hi;
            cen[3 * (size_t)k + a] = 0.5 * ((double)lo + (double)hi);
        }
        perm[k] = k;
    }
    build_ctx ctx = {tlo, thi, cen, perm, tmp, nodes, 0, 2 * n_tris, 0, max_leaf};
    build_rec(&ctx, 0, n_tris, 0);
    *n_nodes_out = ctx.n_nodes;
    *max_depth_out = ctx.max_depth;
    free(tlo); free(thi); free(cen); free(tmp);
    return 0;
}

/* ======================================================================
 * Oracle B part 1a': refit to new vertex positions
 *
 * Not in the paper; defined in words: the topology stays; every box grows
 * from (+inf, -inf) by strict comparisons -- a triangle's over its vertices
 * 0, 1, 2, a leaf's over its triangles in leaf order, an inner node's over its
 * first child's box, then its second's.  A vertex index >= n_vertices reads
 * NaN coordinates, which never pass a strict comparison.
 * ====================================================================== */

/* Grows (lo, hi) by the box (blo, bhi) -- a point when blo == bhi -- with
 * strict comparisons: a bound moves only to a strictly smaller (larger)
 * value, so the first of equal values, and its sign of zero, stays. */
static void grow_strict(float lo[3], float hi[3], const float blo[3], const float bhi[3])
{
    for (int a = 0; a < 3; ++a) {
        if (blo[a] < lo[a]) lo[a] = blo[a];
        if (bhi[a] > hi[a]) hi[a] = bhi[a];
    }
}

/* Recomputes every node box of an oracle BVH (nodes, in place) from the
 * indexed mesh (vertices [n_vertices][3], faces [n_tris][3] by input
 * triangle index); perm maps leaf order to input index.  Node ids are
 * preorder, so children come after their parent and a backward sweep sees
 * them first. */
int orc_refit(orc_node *nodes, uint32_t n_nodes, const uint32_t *perm, uint32_t n_tris,
              const float *vertices, uint32_t n_vertices, const uint32_t *faces)
{
    if (n_tris == 0) return 0;
    for (uint32_t k = n_nodes; k-- > 0;) {
        orc_node *nd = &nodes[k];
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        if (nd->count > 0) {
            for (uint32_t j = nd->first; j < nd->first + nd->count; ++j) {
                const uint32_t prim = perm[j];
                if (prim >= n_tris) return -1;
                for (int c = 0; c < 3; ++c) {
                    const uint32_t vi = faces[3 * (size_t)prim + c];
                    float p[3] = {NAN, NAN, NAN};
                    if (vi < n_vertices)
                        for (int a = 0; a < 3; ++a) p[a] = vertices[3 * (size_t)vi + a];
                    grow_strict(lo, hi, p, p);
                }
            }
        } else {
            grow_strict(lo, hi, nodes[nd->left].lo, nodes[nd->left].hi);
            grow_strict(lo, hi, nodes[nd->right].lo, nodes[nd->right].hi);
        }
        for (int a = 0; a < 3; ++a) {
            nd->lo[a] = lo[a];
            nd->hi[a] = hi[a];
        }
    }
    return 0;
}

/* ======================================================================
 * Oracle B part 1b: the 32-byte node layout (8-bit child boxes)
 *
 * Not in the paper (its BVH format is open); the layout is defined in words:
 * for an inner node with child boxes B0, B1, per axis a
 *   L = min(lo0, lo1), H = max(hi0, hi1);
 *   org = the largest float <= L whose bit pattern has its low 8 bits clear;
 *   E   = the smallest integer in [1, 254] with fma(255, 2^(E-127), org) >= H;
 *   frame word F = bits(org) | E;
 *   decode(q) = fma(q, 2^(E-127), org) for q in 0..255;
 *   qlo = the largest q with decode(q) <= lo, qhi = the smallest q with
 *   decode(q) >= hi, for each child coordinate.
 * Byte order of the twelve q: qlo0.xyz, qhi0.xyz, qlo1.xyz, qhi1.xyz.
 * The traversal decodes the child boxes from F and q and runs the same slab
 * test on them; the root keeps its float32 box.
 * ====================================================================== */

static uint32_t bits_of(float f)
{
    uint32_t b;
    memcpy(&b, &f, 4);
    return b;
}

static float float_of(uint32_t b)
{
    float f;
    memcpy(&f, &b, 4);
    return f;
}

/* The largest float <= L whose pattern has its low 8 bits clear: for L >= 0
 * clearing the bits lowers the value; for L < 0 it would raise it, so the
 * magnitude goes up to the next pattern with clear low bits instead. */
static float frame_origin(float L)
{
    uint32_t b = bits_of(L);
    if (!(b & 0x80000000u) || (b & 0xFFu) == 0) return float_of(b & ~0xFFu);
    return float_of((b | 0xFFu) + 1u);
}

static float q8_decode(uint32_t q, uint32_t frame)
{
    float org = float_of(frame & ~0xFFu);
    float s = float_of((frame & 0xFFu) << 23);
    return fmaf((float)q, s, org);
}

/* Quantizes every inner node of an oracle BVH: frames [n_nodes][3] words,
 * q [n_nodes][12] bytes and the decoded child boxes qbox [n_nodes][12]
 * floats (lo0, hi0, lo1, hi1); leaf entries are zero.  Returns -1 if some
 * axis has no valid exponent (non-finite boxes). */
int orc_quantize(const orc_node *nodes, uint32_t n_nodes, uint32_t *frames, uint8_t *q,
                 float *qbox)
{
    memset(frames, 0, sizeof(uint32_t) * 3 * (size_t)n_nodes);
    memset(q, 0, 12 * (size_t)n_nodes);
    memset(qbox, 0, sizeof(float) * 12 * (size_t)n_nodes);
    for (uint32_t n = 0; n < n_nodes; ++n) {
        const orc_node *nd = &nodes[n];
        if (nd->count > 0) continue;
        const orc_node *ch[2] = {&nodes[nd->left], &nodes[nd->right]};
        for (int a = 0; a < 3; ++a) {
            float L = fminf(ch[0]->lo[a], ch[1]->lo[a]);
            float H = fmaxf(ch[0]->hi[a], ch[1]->hi[a]);
            float org = frame_origin(L);
            uint32_t E = 0;
            for (uint32_t e = 1; e <= 254; ++e) {
                if (fmaf(255.0f, float_of(e << 23), org) >= H) { E = e; break; }
            }
            if (E == 0) return -1;
            uint32_t F = bits_of(org) | E;
            frames[3 * (size_t)n + a] = F;
            for (int c = 0; c < 2; ++c) {
                uint32_t qlo = 0, qhi = 255;
                for (uint32_t k = 256; k-- > 0;)
                    if (q8_decode(k, F) <= ch[c]->lo[a]) { qlo = k; break; }
                for (uint32_t k = 0; k < 256; ++k)
                    if (q8_decode(k, F) >= ch[c]->hi[a]) { qhi = k; break; }
                q[12 * (size_t)n + 6 * c + a] = (uint8_t)qlo;
                q[12 * (size_t)n + 6 * c + 3 + a] = (uint8_t)qhi;
            }
        }
        /* the traversal's boxes come from the stored words alone */
        for (int c = 0; c < 2; ++c)
            for (int a = 0; a < 3; ++a) {
                uint32_t F = frames[3 * (size_t)n + a];
                qbox[12 * (size_t)n + 6 * c + a] = q8_decode(q[12 * (size_t)n + 6 * c + a], F);
                qbox[12 * (size_t)n + 6 * c + 3 + a] = q8_decode(q[12 * (size_t)n + 6 * c + 3 + a], F);
            }
    }
    return 0;
}

/* ======================================================================
 * Oracle B part 1b': the packed-reference layout (48-byte nodes)
 *
 * Not in the paper (it leaves the node format open); defined in words:
 *   words     the twelve child-box words lo0.xyz, hi0.xyz, lo1.xyz, hi1.xyz.
 *   refs      child c's reference -- the index of an inner child among the
 *             inner nodes in depth-first preorder, or count << 29 | first
 *             for a leaf child -- is split into bytes, least significant
 *             first; byte k is the low byte of the bit pattern of the
 *             child's k-th word among lo.x, lo.y, lo.z, hi.x.
 *   moving    each of those four words becomes the nearest float, outward
 *             (down for lo, up for hi), whose pattern has that low byte;
 *             hi.y and hi.z stay.
 * The traversal tests the stored words as the child boxes.
 * ====================================================================== */

/* Walks from x one float at a time (nextafterf, downward for a lower bound,
 * upward for an upper one) until the bit pattern's low byte is `byte`; -1 if
 * the walk reaches an infinity. */
static int move_to_byte(float x, uint32_t byte, int lower, float *out)
{
    float y = x;
    for (int step = 0; step <= 512; ++step) {
        if (isinf(y)) return -1;
        if ((bits_of(y) & 0xFFu) == byte) {
            *out = y;
            return 0;
        }
        y = nextafterf(y, lower ? -INFINITY : INFINITY);
    }
    return -1;
}

/* One word's move, for the tests: 0 and *out, or -1. */
int orc_move_word(float x, uint32_t byte, int lower, float *out)
{
    return move_to_byte(x, byte & 0xFFu, lower, out);
}

/* The packed child boxes pbox [n_nodes][12] (lo0, hi0, lo1, hi1, as stored)
 * and the canonical child references refs [n_nodes][2] of every inner node
 * of an oracle BVH (leaf entries zero).  Returns -1 if a word cannot move. */
int orc_pack(const orc_node *nodes, uint32_t n_nodes, float *pbox, uint32_t *refs)
{
    memset(pbox, 0, sizeof(float) * 12 * (size_t)n_nodes);
    memset(refs, 0, sizeof(uint32_t) * 2 * (size_t)n_nodes);
    uint32_t *inner_index = (uint32_t *)malloc(sizeof(uint32_t) * (n_nodes ? n_nodes : 1));
    if (!inner_index) return -2;
    uint32_t k = 0;
    for (uint32_t n = 0; n < n_nodes; ++n)  /* node ids are preorder */
        inner_index[n] = nodes[n].count == 0 ? k++ : 0;
    for (uint32_t n = 0; n < n_nodes; ++n) {
        const orc_node *nd = &nodes[n];
        if (nd->count > 0) continue;
        const uint32_t child[2] = {nd->left, nd->right};
        for (int c = 0; c < 2; ++c) {
            const orc_node *ch = &nodes[child[c]];
            const uint32_t ref = ch->count > 0 ? (ch->count << 29 | ch->first) : inner_index[child[c]];
            refs[2 * (size_t)n + c] = ref;
            float *b = pbox + 12 * (size_t)n + 6 * c;
            for (int a = 0; a < 3; ++a) {
                b[a] = ch->lo[a];
                b[3 + a] = ch->hi[a];
            }
            /* bytes 0..2 into lo.x, lo.y, lo.z; byte 3 into hi.x */
            for (int j = 0; j < 4; ++j) {
                const int w = j < 3 ? j : 3;
                if (move_to_byte(b[w], (ref >> (8 * j)) & 0xFFu, j < 3, &b[w]) != 0) {
                    free(inner_index);
                    return -1;
                }
            }
        }
    }
    free(inner_index);
    return 0;
}

/* ======================================================================
 * Oracle B part 1c: the four-wide layout
 *
 * Not in the paper (it leaves the BVH's arity open); defined in words:
 *   collapse  for a binary inner node X the child list starts [X.left,
 *             X.right]; while it has fewer than 4 entries and one of them is
 *             a binary inner node, the inner entry with the largest box
 *             surface area (float64; ties -> the earliest in the list) is
 *             replaced at its place by its left child followed by its right
 *             child.  Inner entries of the final list head wide nodes of
 *             their own; leaf entries are the binary leaves.
 *   traverse at a wide node with k children, box-test children 0..k-1 in
 *             order (each counted); order the hit ones by (tn, child index)
 *             ascending, visit the first and push the others from the last to
 *             the second (the second ends on top); none hit -> pop.  Pops,
 *             leaves and counting as in the binary traversal.
 *   bound     the stack never holds more than the largest sum of (k - 1)
 *             over the wide nodes of a root-to-leaf path.
 * The oracle keys each wide node by the index of the binary node heading it.
 * ====================================================================== */

typedef struct {
    uint32_t n;         /* children (2..4); 0 if this binary node heads no wide node */
    uint32_t child[4];  /* binary node indices, in list order */
} orc_wide;

static uint32_t widen_rec(const orc_node *nodes, uint32_t x, orc_wide *wide, uint32_t *order,
                          uint32_t *n_order, uint32_t *bound)
{
    uint32_t list[4] = {nodes[x].left, nodes[x].right, 0, 0};
    uint32_t n = 2;
    while (n < 4) {
        int best = -1;
        double best_area = -1.0;
        for (uint32_t i = 0; i < n; ++i) {
            const orc_node *c = &nodes[list[i]];
            if (c->count != 0) continue;
            double a = box_area(c->lo, c->hi);
            if (a > best_area) { best_area = a; best = (int)i; }
        }
        if (best < 0) break;
        uint32_t y = list[best];
        for (uint32_t i = n; i > (uint32_t)best + 1; --i) list[i] = list[i - 1];
        list[best] = nodes[y].left;
        list[best + 1] = nodes[y].right;
        ++n;
    }
    wide[x].n = n;
    for (uint32_t i = 0; i < 4; ++i) wide[x].child[i] = i < n ? list[i] : 0;
    order[(*n_order)++] = x;
    uint32_t count = 1, deepest = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (nodes[list[i]].count != 0) continue;
        uint32_t b = 0;
        count += widen_rec(nodes, list[i], wide, order, n_order, &b);
        if (b > deepest) deepest = b;
    }
    *bound = (n - 1) + deepest;
    return count;
}

/* Collapses an oracle BVH (n_nodes binary nodes, node 0 the root) into the
 * four-wide layout.  wide[] has n_nodes entries (keyed by binary index);
 * order[] receives the heads of the wide nodes in depth-first preorder
 * (children in list order).  Outputs the wide node count and the stack
 * bound; a root that is a leaf (or an empty scene) gives none. */
int orc_widen(const orc_node *nodes, uint32_t n_nodes, orc_wide *wide, uint32_t *order,
              uint32_t *n_wide, uint32_t *stack_bound)
{
    for (uint32_t i = 0; i < n_nodes; ++i) memset(&wide[i], 0, sizeof wide[i]);
    *n_wide = 0;
    *stack_bound = 0;
    if (n_nodes == 0 || nodes[0].count != 0 || n_nodes == 1) return 0;
    uint32_t n_order = 0;
    *n_wide = widen_rec(nodes, 0, wide, order, &n_order, stack_bound);
    return n_order == *n_wide ? 0 : -1;
}

/* ======================================================================
 * Oracle B part 2: float32 while-while traversal (Algorithm 1)
 *
 * Per ray:
 *   setup   d' = d with components of magnitude < 2^-80 replaced by
 *           +-2^-80; inv = 1/d'; ood = o*inv; tmax_cur = tmax.
 *   box     t0 = fma(lo, inv, -ood), t1 = fma(hi, inv, -ood) per axis;
 *           tn = max(max(max(min x, min y), min z), tmin),
 *           tf = min(min(min(max x, max y), max z), tmax_cur); hit iff tn <= tf.
 *           Every box test is counted.
 *   root    test the root box; a miss ends the ray.
 *   inner   test both children's boxes; both hit -> visit the one with the
 *           smaller tn (tie -> left) and push the other with its tn; one hit ->
 *           visit it; none -> pop.
 *   pop     discard entries whose tn > tmax_cur; an empty stack ends the ray.
 *   leaf    test the leaf's triangles in stored order (each counted), then pop.
 *   tri     Moller-Trumbore, two-sided: p = d x e2, det = e1.p, det == 0 ->
 *           no hit; r = 1/det; s = o - v0; u = (s.p) r, reject unless
 *           0 <= u <= 1; q = s x e1; v = (d.q) r, reject unless v >= 0 and
 *           u + v <= 1; t = (e2.q) r, candidate iff tmin < t < tmax_cur, with
 *           e1 = v1 - v0, e2 = v2 - v0 rounded to float32,
 *           dot(a,b) = fma(a.z,b.z, fma(a.y,b.y, a.x*b.x)) and
 *           cross(a,b)_x = fma(a.y,b.z, -(a.z*b.y)) (cyclically).
 *           A candidate is handed to the intersector (counted); if accepted:
 *           closest-hit -> tmax_cur = t and the record is kept; any-hit -> stop.
 *   alpha   w0 = (1-u)-v; s = fma(v,tc2, fma(u,tc1, w0*tc0)) per coordinate;
 *           x = clamp(floor(s*W), 0, W-1), y likewise from t and H;
 *           accept iff texel(geom, y, x) >> 24 >= alpha_min.
 *   checker accept iff floor(n*u) + floor(n*v) is even.
 * ====================================================================== */

typedef struct {
    const float *verts;
    const uint32_t *geom;
    uint32_t n_tris;
    const orc_node *nodes;
    const uint32_t *perm;
    uint32_t n_nodes;
    const float *rays;
    uint32_t n_rays;
    int kind;
    orc_isect is;
    int any_hit;
    uint32_t multi_k;   /* > 0: multi-hit query keeping the multi_k nearest */
    float *t, *u, *v;   /* [n_rays] or, for multi-hit, [n_rays][multi_k] */
    uint32_t *prim;
    uint32_t *n_hits;   /* multi-hit: hits found per ray */
    uint32_t *counters; /* [n_rays][4]: boxes, triangles, candidates, accepts */
    const float *qbox;  /* 32-byte layout: decoded child boxes per node, or NULL */
    const orc_wide *wide; /* four-wide layout (by binary head index), or NULL */
    uint32_t next;
    pthread_mutex_t lock;
} trav_job;

static float dot3f(const float a[3], const float b[3])
{
    return fmaf(a[2], b[2], fmaf(a[1], b[1], a[0] * b[0]));
}

static void cross3f(const float a[3], const float b[3], float r[3])
{
    r[0] = fmaf(a[1], b[2], -(a[2] * b[1]));
    r[1] = fmaf(a[2], b[0], -(a[0] * b[2]));
    r[2] = fmaf(a[0], b[1], -(a[1] * b[0]));
}

typedef struct {
    float o[3], d[3], inv[3], ood[3];
    float tmin, tmax_cur;
    /* record */
    float t, u, v;
    uint32_t prim;
    int done;
    /* multi-hit list, sorted by t (ties: earlier accepted first) */
    uint32_t k, n;
    float tmax0;
    float lt[ORC_MAX_MULTI], lu[ORC_MAX_MULTI], lv[ORC_MAX_MULTI];
    uint32_t lp[ORC_MAX_MULTI];
    uint32_t n_box, n_tri, n_cand, n_acc;
} ray_state;

/* Box test (the intersect(ray, aabb) call site of Algorithm 1); the counter
 * is the heat-map intersector's interception of that call. */
static int box_test(ray_state *rs, const float lo[3], const float hi[3], float *tn_out)
{
    rs->n_box++;
    float t0[3], t1[3];
    for (int a = 0; a < 3; ++a) {
        t0[a] = fmaf(lo[a], rs->inv[a], -rs->ood[a]);
        t1[a] = fmaf(hi[a], rs->inv[a], -rs->ood[a]);
    }
    float tn = fmaxf(fmaxf(fmaxf(fminf(t0[0], t1[0]), fminf(t0[1], t1[1])), fminf(t0[2], t1[2])), rs->tmin);
    float tf = fminf(fminf(fminf(fmaxf(t0[0], t1[0]), fmaxf(t0[1], t1[1])), fmaxf(t0[2], t1[2])), rs->tmax_cur);
    *tn_out = tn;
    return tn <= tf;
}

static int accept32(const trav_job *job, uint32_t prim, float u, float v)
{
    if (job->kind == ORC_ALPHA) {
        const orc_isect *is = &job->is;
        const float *tc = is->texcoords + (size_t)prim * 6;
        float w0 = (1.0f - u) - v;
        float s = fmaf(v, tc[4], fmaf(u, tc[2], w0 * tc[0]));
        float t = fmaf(v, tc[5], fmaf(u, tc[3], w0 * tc[1]));
        float xf = floorf(s * (float)is->width);
        float yf = floorf(t * (float)is->height);
        if (xf < 0.0f) xf = 0.0f;
        if (xf > (float)(is->width - 1)) xf = (float)(is->width - 1);
        if (yf < 0.0f) yf = 0.0f;
        if (yf > (float)(is->height - 1)) yf = (float)(is->height - 1);
        uint32_t g = job->geom ? job->geom[prim] : 0;
        uint32_t texel = is->textures[((size_t)g * is->height + (uint32_t)yf) * is->width + (uint32_t)xf];
        return (texel >> 24) >= is->alpha_min;
    }
    if (job->kind == ORC_PROCEDURAL) {
        float n = (float)job->is.checker_n;
        int a = (int)floorf(n * u), b = (int)floorf(n * v);
        return ((a + b) & 1) == 0;
    }
    return 1;
}

/* Triangle test (the intersect(ray, prim) call site) followed by the
 * intersector's decision. */
static void tri_test(const trav_job *job, ray_state *rs, uint32_t slot)
{
    rs->n_tri++;
    uint32_t prim = job->perm[slot];
    const float *tv = job->verts + 9 * (size_t)prim;
    float v0[3] = {tv[0], tv[1], tv[2]};
    float e1[3] = {tv[3] - tv[0], tv[4] - tv[1], tv[5] - tv[2]};
    float e2[3] = {tv[6] - tv[0], tv[7] - tv[1], tv[8] - tv[2]};
    float p[3], q[3], s[3];
    cross3f(rs->d, e2, p);
    float det = dot3f(e1, p);
    if (det == 0.0f) return;
    float r = 1.0f / det;
    s[0] = rs->o[0] - v0[0]; s[1] = rs->o[1] - v0[1]; s[2] = rs->o[2] - v0[2];
    float u = dot3f(s, p) * r;
    if (!(u >= 0.0f && u <= 1.0f)) return;
    cross3f(s, e1, q);
    float v = dot3f(rs->d, q) * r;
    if (!(v >= 0.0f && u + v <= 1.0f)) return;
    float t = dot3f(e2, q) * r;
    if (!(t > rs->tmin && t < rs->tmax_cur)) return;
    rs->n_cand++;
    if (!accept32(job, prim, u, v)) return;
    rs->n_acc++;
    if (rs->k > 0) {
        /* multi-hit: insert after every kept hit with t' <= t; the k-th
         * nearest distance, once k hits are kept, bounds the search */
        uint32_t pos = rs->n;
        while (pos > 0 && t < rs->lt[pos - 1]) --pos;
        if (pos >= rs->k) return;
        uint32_t last = rs->n < rs->k ? rs->n : rs->k - 1;
        for (uint32_t i = last; i > pos; --i) {
            rs->lt[i] = rs->lt[i - 1]; rs->lu[i] = rs->lu[i - 1];
            rs->lv[i] = rs->lv[i - 1]; rs->lp[i] = rs->lp[i - 1];
        }
        rs->lt[pos] = t; rs->lu[pos] = u; rs->lv[pos] = v; rs->lp[pos] = prim;
        if (rs->n < rs->k) rs->n++;
        if (rs->n == rs->k) rs->tmax_cur = rs->lt[rs->k - 1] < rs->tmax0 ? rs->lt[rs->k - 1] : rs->tmax0;
        return;
    }
    rs->prim = prim;
    rs->t = t; rs->u = u; rs->v = v;
    if (job->any_hit) rs->done = 1;
    else rs->tmax_cur = t;
}

static void trav_one(trav_job *job, uint32_t i)
{
    const float *r = job->rays + (size_t)i * 8;
    ray_state rs;
    memset(&rs, 0, sizeof rs);
    const float tiny = 0x1p-80f;
    for (int a = 0; a < 3; ++a) {
        rs.o[a] = r[a];
        rs.d[a] = r[4 + a];
        float dd = rs.d[a];
        if (fabsf(dd) < tiny) dd = copysignf(tiny, dd);
        rs.inv[a] = 1.0f / dd;
        rs.ood[a] = rs.o[a] * rs.inv[a];
    }
    rs.tmin = r[3];
    rs.tmax_cur = r[7];
    rs.tmax0 = r[7];
    rs.prim = ORC_MISS;
    rs.t = INFINITY;
    rs.k = job->multi_k;

    if (job->n_tris > 0) {
        uint32_t stack_node[128];
        float stack_tn[128];
        int sp = 0;
        float tn;
        uint32_t cur = 0;
        int alive = box_test(&rs, job->nodes[0].lo, job->nodes[0].hi, &tn);
        while (alive && !rs.done) {
            /* descend through inner nodes */
            while (job->wide && job->nodes[cur].count == 0) {
                const orc_wide *w = &job->wide[cur];
                float tn4[4];
                uint32_t hits[4], m = 0;
                for (uint32_t c = 0; c < w->n; ++c) {
                    const orc_node *ch = &job->nodes[w->child[c]];
                    if (!box_test(&rs, ch->lo, ch->hi, &tn4[c])) continue;
                    /* insert c after every hit child with tn <= tn4[c] */
                    uint32_t pos = m;
                    while (pos > 0 && tn4[c] < tn4[hits[pos - 1]]) { hits[pos] = hits[pos - 1]; --pos; }
                    hits[pos] = c;
                    ++m;
                }
                if (m > 0) {
                    for (uint32_t j = m - 1; j >= 1; --j) {
                        stack_node[sp] = w->child[hits[j]];
                        stack_tn[sp] = tn4[hits[j]];
                        ++sp;
                    }
                    cur = w->child[hits[0]];
                } else {
                    alive = 0;
                    while (sp > 0) {
                        --sp;
                        if (!(stack_tn[sp] > rs.tmax_cur)) { cur = stack_node[sp]; alive = 1; break; }
                    }
                    if (!alive) break;
                }
            }
            while (!job->wide && job->nodes[cur].count == 0) {
                const orc_node *nd = &job->nodes[cur];
                float tl, tr;
                int hl, hr;
                if (job->qbox) {
                    const float *qb = job->qbox + 12 * (size_t)cur;
                    hl = box_test(&rs, qb, qb + 3, &tl);
                    hr = box_test(&rs, qb + 6, qb + 9, &tr);
                } else {
                    hl = box_test(&rs, job->nodes[nd->left].lo, job->nodes[nd->left].hi, &tl);
                    hr = box_test(&rs, job->nodes[nd->right].lo, job->nodes[nd->right].hi, &tr);
                }
                if (hl && hr) {
                    if (tr < tl) { cur = nd->right; stack_node[sp] = nd->left; stack_tn[sp] = tl; }
                    else { cur = nd->left; stack_node[sp] = nd->right; stack_tn[sp] = tr; }
                    ++sp;
                } else if (hl) {
                    cur = nd->left;
                } else if (hr) {
                    cur = nd->right;
                } else {
                    alive = 0;
                    while (sp > 0) {
                        --sp;
                        if (!(stack_tn[sp] > rs.tmax_cur)) { cur = stack_node[sp]; alive = 1; break; }
                    }
                    if (!alive) break;
                }
            }
            if (!alive) break;
            /* leaf: test its triangles in stored order */
            const orc_node *lf = &job->nodes[cur];
            for (uint32_t j = lf->first; j < lf->first + lf->count && !rs.done; ++j)
                tri_test(job, &rs, j);
            if (rs.done) break;
            alive = 0;
            while (sp > 0) {
                --sp;
                if (!(stack_tn[sp] > rs.tmax_cur)) { cur = stack_node[sp]; alive = 1; break; }
            }
        }
    }

    if (job->multi_k > 0) {
        for (uint32_t j = 0; j < job->multi_k; ++j) {
            size_t o = (size_t)i * job->multi_k + j;
            int kept = j < rs.n;
            job->t[o] = kept ? rs.lt[j] : INFINITY;
            job->u[o] = kept ? rs.lu[j] : 0.0f;
            job->v[o] = kept ? rs.lv[j] : 0.0f;
            job->prim[o] = kept ? rs.lp[j] : ORC_MISS;
        }
        job->n_hits[i] = rs.n;
    } else {
        if (rs.prim == ORC_MISS) { rs.t = INFINITY; rs.u = 0.0f; rs.v = 0.0f; }
        job->t[i] = rs.t;
        job->u[i] = rs.u;
        job->v[i] = rs.v;
        job->prim[i] = rs.prim;
    }
    if (job->counters) {
        uint32_t *c = job->counters + 4 * (size_t)i;
        c[0] = rs.n_box; c[1] = rs.n_tri; c[2] = rs.n_cand; c[3] = rs.n_acc;
    }
}

static void *trav_worker(void *arg)
{
    trav_job *job = (trav_job *)arg;
    for (;;) {
        pthread_mutex_lock(&job->lock);
        uint32_t b = job->next;
        job->next = b + 256 < job->n_rays ? b + 256 : job->n_rays;
        uint32_t e = job->next;
        pthread_mutex_unlock(&job->lock);
        if (b >= e) break;
        for (uint32_t i = b; i < e; ++i) trav_one(job, i);
    }
    return NULL;
}

/* Oracle B traversal over a BVH made by orc_build.  Outputs t/u/v/prim per
 * ray (misses: prim = ORC_MISS, t = +inf, u = v = 0; any-hit: the first
 * accepted hit; multi-hit (multi_k > 0): the multi_k nearest accepted hits in
 * increasing t, ties in acceptance order, padded with misses, and their number
 * in n_hits) and, if counters != NULL, four uint32 counters per ray. */
int orc_traverse_layout(const float *verts, const uint32_t *geom_ids, uint32_t n_tris,
                        const orc_node *nodes, const uint32_t *perm, uint32_t n_nodes,
                        const float *qbox, const float *rays, uint32_t n_rays, int kind,
                        const orc_isect *is, int any_hit, uint32_t multi_k, float *t,
                        uint32_t *prim, float *u, float *v, uint32_t *n_hits, uint32_t *counters,
                        int n_threads);

/* The traversal over the four-wide layout of the same BVH (wide from
 * orc_widen; the binary nodes supply the boxes and the leaves). */
int orc_traverse_wide(const float *verts, const uint32_t *geom_ids, uint32_t n_tris,
                      const orc_node *nodes, const uint32_t *perm, uint32_t n_nodes,
                      const orc_wide *wide, const float *rays, uint32_t n_rays, int kind,
                      const orc_isect *is, int any_hit, uint32_t multi_k, float *t,
                      uint32_t *prim, float *u, float *v, uint32_t *n_hits, uint32_t *counters,
                      int n_threads);

int orc_traverse(const float *verts, const uint32_t *geom_ids, uint32_t n_tris,
                 const orc_node *nodes, const uint32_t *perm, uint32_t n_nodes,
                 const float *rays, uint32_t n_rays, int kind, const orc_isect *is,
                 int any_hit, uint32_t multi_k, float *t, uint32_t *prim, float *u, float *v,
                 uint32_t *n_hits, uint32_t *counters, int n_threads)
{
    return orc_traverse_layout(verts, geom_ids, n_tris, nodes, perm, n_nodes, NULL, rays, n_rays,
                               kind, is, any_hit, multi_k, t, prim, u, v, n_hits, counters,
                               n_threads);
}

/* The same traversal; with qbox (orc_quantize's decoded child boxes, or
 * orc_pack's stored ones) the inner nodes' box tests use that layout's
 * boxes. */
int orc_traverse_layout(const float *verts, const uint32_t *geom_ids, uint32_t n_tris,
                        const orc_node *nodes, const uint32_t *perm, uint32_t n_nodes,
                        const float *qbox, const float *rays, uint32_t n_rays, int kind,
                        const orc_isect *is, int any_hit, uint32_t multi_k, float *t,
                        uint32_t *prim, float *u, float *v, uint32_t *n_hits, uint32_t *counters,
                        int n_threads)
{
    if (kind < ORC_DEFAULT || kind > ORC_PROCEDURAL) return -1;
    if (multi_k > ORC_MAX_MULTI || (multi_k > 0 && (any_hit || !n_hits))) return -2;
    trav_job job;
    memset(&job, 0, sizeof job);
    job.verts = verts; job.geom = geom_ids; job.n_tris = n_tris;
    job.nodes = nodes; job.perm = perm; job.n_nodes = n_nodes;
    job.rays = rays; job.n_rays = n_rays; job.kind = kind;
    if (is) job.is = *is;
    job.any_hit = any_hit;
    job.multi_k = multi_k;
    job.t = t; job.u = u; job.v = v; job.prim = prim; job.counters = counters;
    job.n_hits = n_hits;
    job.qbox = qbox;
    pthread_mutex_init(&job.lock, NULL);
    run_threads(trav_worker, &job, n_threads);
    pthread_mutex_destroy(&job.lock);
    return 0;
}

int orc_traverse_wide(const float *verts, const uint32_t *geom_ids, uint32_t n_tris,
                      const orc_node *nodes, const uint32_t *perm, uint32_t n_nodes,
                      const orc_wide *wide, const float *rays, uint32_t n_rays, int kind,
                      const orc_isect *is, int any_hit, uint32_t multi_k, float *t,
                      uint32_t *prim, float *u, float *v, uint32_t *n_hits, uint32_t *counters,
                      int n_threads)
{
    if (kind < ORC_DEFAULT || kind > ORC_PROCEDURAL) return -1;
    if (multi_k > ORC_MAX_MULTI || (multi_k > 0 && (any_hit || !n_hits))) return -2;
    if (!wide) return -3;
    trav_job job;
    memset(&job, 0, sizeof job);
    job.verts = verts; job.geom = geom_ids; job.n_tris = n_tris;
    job.nodes = nodes; job.perm = perm; job.n_nodes = n_nodes;
    job.rays = rays; job.n_rays = n_rays; job.kind = kind;
    if (is) job.is = *is;
    job.any_hit = any_hit;
    job.multi_k = multi_k;
    job.t = t; job.u = u; job.v = v; job.prim = prim; job.counters = counters;
    job.n_hits = n_hits;
    job.wide = wide;
    pthread_mutex_init(&job.lock, NULL);
    run_threads(trav_worker, &job, n_threads);
    pthread_mutex_destroy(&job.lock);
    return 0;
}

uint32_t orc_node_size(void) { return (uint32_t)sizeof(orc_node); }

/* ======================================================================
 * Gradient of the accepted hit (differentiable closest hit)
 *
 * For a ray that hit triangle (v0, v1, v2) at (t, u, v), the hit point
 * satisfies F = o + t d - (1-u-v) v0 - u v1 - v v2 = 0.  With A = dF/d(t,u,v)
 * = [d, -e1, -e2] (columns; e1 = v1 - v0, e2 = v2 - v0) the implicit function
 * theorem gives d(t,u,v) = -A^-1 dF, so for an upstream gradient
 * g = (dL/dt, dL/du, dL/dv):  dL/dtheta = lam . dF/dtheta with
 * lam = -A^-T g, i.e.
 *   dL/do = lam, dL/dd = t lam, dL/dv0 = -(1-u-v) lam, dL/dv1 = -u lam,
 *   dL/dv2 = -v lam.
 * A^T lam = -g reads d.lam = -g_t, e1.lam = g_u, e2.lam = g_v, solved here
 * with the scalar triple product: lam = (-g_t (e1 x e2) + g_u (e2 x d)
 * + g_v (d x e1)) / (d . (e1 x e2)).  The hit prim stays fixed and the
 * intersector's decision is not differentiated (it is discrete).
 * ====================================================================== */

/* float64 (t, u, v) of ray i against the fixed triangle faces[prims[i]] of
 * the float64 vertex array (plane formulation, no inside test); rays with
 * prim = ORC_MISS or a parallel triangle get NaN. */
int orc_fixed_hit64(const double *verts, const uint32_t *faces, const float *rays,
                    const uint32_t *prims, uint32_t n_rays, double *tuv)
{
    for (uint32_t i = 0; i < n_rays; ++i) {
        double *out = tuv + 3 * (size_t)i;
        out[0] = out[1] = out[2] = NAN;
        if (prims[i] == ORC_MISS) continue;
        const float *r = rays + 8 * (size_t)i;
        d3 o = {r[0], r[1], r[2]}, d = {r[4], r[5], r[6]};
        const uint32_t *f = faces + 3 * (size_t)prims[i];
        d3 v0 = {verts[3 * f[0]], verts[3 * f[0] + 1], verts[3 * f[0] + 2]};
        d3 v1 = {verts[3 * f[1]], verts[3 * f[1] + 1], verts[3 * f[1] + 2]};
        d3 v2 = {verts[3 * f[2]], verts[3 * f[2] + 1], verts[3 * f[2] + 2]};
        d3 e1 = d3_sub(v1, v0), e2 = d3_sub(v2, v0);
        d3 nrm = d3_cross(e1, e2);
        double dn = d3_dot(d, nrm);
        if (dn == 0.0) continue;
        double t = d3_dot(d3_sub(v0, o), nrm) / dn;
        d3 w = d3_sub(d3_add(o, d3_scale(d, t)), v0);
        double nn = d3_dot(nrm, nrm);
        out[0] = t;
        out[1] = d3_dot(d3_cross(w, e2), nrm) / nn;
        out[2] = d3_dot(d3_cross(e1, w), nrm) / nn;
    }
    return 0;
}

/* float64 closed-form gradient.  grad_verts [n_verts][3] is accumulated
 * (caller zeroes it); grad_rays [n_rays][6] (dL/do, dL/dd) is overwritten
 * (zero for misses).  (t, u, v) are recomputed in float64 for the fixed
 * prim. */
int orc_hit_grad64(const double *verts, uint32_t n_verts, const uint32_t *faces,
                   const float *rays, const uint32_t *prims, const double *grad_tuv,
                   uint32_t n_rays, double *grad_verts, double *grad_rays)
{
    for (uint32_t i = 0; i < n_rays; ++i) {
        double *gr = grad_rays ? grad_rays + 6 * (size_t)i : NULL;
        if (gr) for (int k = 0; k < 6; ++k) gr[k] = 0.0;
        if (prims[i] == ORC_MISS) continue;
        double tuv[3];
        orc_fixed_hit64(verts, faces, rays + 8 * (size_t)i, prims + i, 1, tuv);
        if (isnan(tuv[0])) continue;
        const float *r = rays + 8 * (size_t)i;
        d3 d = {r[4], r[5], r[6]};
        const uint32_t *f = faces + 3 * (size_t)prims[i];
        if (f[0] >= n_verts || f[1] >= n_verts || f[2] >= n_verts) return -1;
        d3 v0 = {verts[3 * f[0]], verts[3 * f[0] + 1], verts[3 * f[0] + 2]};
        d3 v1 = {verts[3 * f[1]], verts[3 * f[1] + 1], verts[3 * f[1] + 2]};
        d3 v2 = {verts[3 * f[2]], verts[3 * f[2] + 1], verts[3 * f[2] + 2]};
        d3 e1 = d3_sub(v1, v0), e2 = d3_sub(v2, v0);
        double det = d3_dot(d, d3_cross(e1, e2));
        const double *g = grad_tuv + 3 * (size_t)i;
        d3 lam = d3_add(d3_add(d3_scale(d3_cross(e1, e2), -g[0]), d3_scale(d3_cross(e2, d), g[1])),
                        d3_scale(d3_cross(d, e1), g[2]));
        lam = d3_scale(lam, 1.0 / det);
        double t = tuv[0], u = tuv[1], v = tuv[2], w0 = 1.0 - u - v;
        double c[3] = {-w0, -u, -v};
        for (int k = 0; k < 3; ++k) {
            double *gv = grad_verts + 3 * (size_t)f[k];
            gv[0] += c[k] * lam.x;
            gv[1] += c[k] * lam.y;
            gv[2] += c[k] * lam.z;
        }
        if (gr) {
            gr[0] = lam.x; gr[1] = lam.y; gr[2] = lam.z;
            gr[3] = t * lam.x; gr[4] = t * lam.y; gr[5] = t * lam.z;
        }
    }
    return 0;
}


/* ======================================================================
 * Multi-hit query, float64 definition (Section 3.1: a query returning several hit
 * points, read as the N nearest accepted hits in increasing distance).
 * ====================================================================== */
typedef struct {
    double t, u, v;
    uint32_t k;
} acc_hit;

static int acc_cmp(const void *a, const void *b)
{
    const acc_hit *x = (const acc_hit *)a, *y = (const acc_hit *)b;
    if (x->t < y->t) return -1;
    if (x->t > y->t) return 1;
    return x->k < y->k ? -1 : (x->k > y->k);
}

/* For each ray: every accepted hit, sorted by (t, index); the first K are
 * written ([n_rays][K], padded with misses) with their count.  flags marks
 * rays whose kept set is ambiguous in float32: two accepted distances among
 * the first K+1 within 1e-6 relative (or within their float32 bounds), or a
 * candidate no farther than the K-th kept hit (all candidates when fewer than
 * K were found) that is near an edge or near its filter decision. */
int orc_brute_multi(const float *verts, const uint32_t *geom_ids, uint32_t n_tris,
                    const float *rays, uint32_t n_rays, int kind, const orc_isect *is,
                    uint32_t K, double *t, uint32_t *prim, double *u, double *v,
                    uint32_t *n_hits, uint8_t *flags, int n_threads)
{
    (void)n_threads;
    if (K == 0 || kind < ORC_DEFAULT || kind > ORC_PROCEDURAL) return -1;
    acc_hit *buf = malloc(sizeof(acc_hit) * (n_tris ? n_tris : 1));
    double *bt = malloc(sizeof(double) * (n_tris ? n_tris : 1));
    if (!buf || !bt) { free(buf); free(bt); return -1; }
    brute_job tmp;
    memset(&tmp, 0, sizeof tmp);
    if (is) tmp.is = *is;
    for (uint32_t i = 0; i < n_rays; ++i) {
        const float *r = rays + 8 * (size_t)i;
        d3 o = {r[0], r[1], r[2]}, d = {r[4], r[5], r[6]};
        double tmin = r[3], tmax = r[7];
        uint32_t m = 0;
        for (uint32_t k = 0; k < n_tris; ++k) {
            double tt, uu, vv, mg, bu, btt;
            if (!plane_hit64(o, d, verts + 9 * (size_t)k, &tt, &uu, &vv, &mg, &bu, &btt)) continue;
            if (!(mg >= 0.0) || !(tt > tmin) || !(tt < tmax)) continue;
            int acc = 1;
            double fm;
            uint32_t g = geom_ids ? geom_ids[k] : 0;
            if (kind == ORC_ALPHA) acc = alpha_accept64(&tmp.is, k, g, uu, vv);
            else if (kind == ORC_PROCEDURAL) acc = checker_accept64(&tmp.is, uu, vv, &fm);
            if (!acc) continue;
            buf[m].t = tt; buf[m].u = uu; buf[m].v = vv; buf[m].k = k;
            bt[m] = btt;
            ++m;
        }
        qsort(buf, m, sizeof(acc_hit), acc_cmp);
        uint32_t keep = m < K ? m : K;
        uint8_t fl = 0;
        for (uint32_t j = 0; j < K; ++j) {
            size_t o2 = (size_t)i * K + j;
            t[o2] = j < keep ? buf[j].t : INFINITY;
            u[o2] = j < keep ? buf[j].u : 0.0;
            v[o2] = j < keep ? buf[j].v : 0.0;
            prim[o2] = j < keep ? buf[j].k : ORC_MISS;
        }
        n_hits[i] = keep;
        uint32_t lim = m < K + 1 ? m : K + 1;
        for (uint32_t j = 1; j < lim; ++j)
            if (buf[j].t - buf[j - 1].t < 1e-6 * fabs(buf[j].t)) fl |= ORC_E_NEAR_TIE;
        double reach = (m >= K) ? buf[K - 1].t * (1.0 + 1e-6) : tmax;
        for (uint32_t k = 0; k < n_tris; ++k) {
            double tt, uu, vv, mg, bu, btt;
            if (!plane_hit64(o, d, verts + 9 * (size_t)k, &tt, &uu, &vv, &mg, &bu, &btt)) continue;
            if (!(tt > tmin - btt) || !(tt < tmax + btt) || !(tt <= reach + btt)) continue;
            double delta = bu > 1e-6 ? bu : 1e-6;
            if (fabs(mg) < delta) fl |= ORC_E_NEAR_EDGE;
            if (mg > -delta && kind == ORC_ALPHA) {
                double wh = tmp.is.width > tmp.is.height ? tmp.is.width : tmp.is.height;
                if (alpha_decision_fragile(&tmp.is, k, geom_ids ? geom_ids[k] : 0, uu, vv,
                                           (2.0 * delta + 0x1p-20) * wh))
                    fl |= ORC_E_NEAR_FILTER;
            } else if (mg > -delta && kind == ORC_PROCEDURAL) {
                double fm;
                checker_accept64(&tmp.is, uu, vv, &fm);
                if (fm < 2.0 * delta * tmp.is.checker_n) fl |= ORC_E_NEAR_FILTER;
            }
            /* a near-equal distance to a kept hit makes the order ambiguous */
            for (uint32_t j = 0; j < keep; ++j)
                if (buf[j].k != k && mg > -delta && fabs(tt - buf[j].t) <= btt + bt[j])
                    fl |= ORC_E_NEAR_TIE;
        }
        flags[i] = fl;
    }
    free(buf);
    free(bt);
    return 0;
}

/* ======================================================================
 * Instancing (Section 3.2: a BVH may itself be a primitive of a BVH; object
 * instancing stores BVHs as the primitives of a top-level BVH).
 *
 * An instance is a bottom-level BVH (blas) plus a row-major 3x4 affine map M
 * from world to object space; a world ray o + t d becomes the object ray
 * M(o) + t L(d) (L = linear part), so the distance t and the barycentrics of
 * a hit are the same in both spaces.  Reading used for the float32 traversal:
 *   o'_i = fma(m_i0, o_x, fma(m_i1, o_y, fma(m_i2, o_z, m_i3)))
 *   d'_i = fma(m_i0, d_x, fma(m_i1, d_y, m_i2 * d_z))
 * The top-level BVH is the binned-SAH BVH over the instances' world boxes
 * (each box given as the degenerate triangle lo, hi, hi); at a top-level leaf
 * the leaf's instances are entered in stored order, each by a full
 * traversal of its bottom-level BVH (root box test in object space first)
 * with the shared distance bound, before the top-level stack is popped.
 * The intersector decides per mesh: the alpha mask (Section 4, Listing 5)
 * reads the hit mesh's own texture coordinates and texture ids, from one
 * texture array shared by all meshes.
 * ====================================================================== */

typedef struct {
    const float *verts;       /* [n_tris][3][3] object space */
    uint32_t n_tris;
    const orc_node *nodes;
    const uint32_t *perm;
    const uint32_t *geom;     /* alpha: texture id per triangle (NULL: 0) */
    const float *texcoords;   /* alpha: [n_tris][3][2] of this mesh */
} orc_blas;

typedef struct {
    uint32_t blas;
    float m[12];              /* object_from_world, row-major 3x4 */
} orc_inst;

/* float64 definition: every instance, every triangle (object-space test of
 * the object-space ray, computed in float64 from the float32 inputs). */
/* Extra float32 error of a hit reached through a float32 object ray.  The
 * traversal forms o' and d' with three roundings per component, so
 * |o'_i - o_i| <= c (|m_i0 o_x| + |m_i1 o_y| + |m_i2 o_z| + |m_i3|) and
 * |d'_i - d_i| <= c (|m_i0 d_x| + |m_i1 d_y| + |m_i2 d_z|), c = 4 eps (above
 * the 3 eps + O(eps^2) of three roundings).  A hit solves
 * o + t d = v0 + u e1 + v e2; perturbing o by do and d by dd moves the
 * solution by [d, -e1, -e2]^-1 (-(do + t dd)), so by Cramer's rule, with
 * w = do + t dd and det = d.(e1 x e2):
 *   |dt| <= |w| |e1 x e2| / |det|,  |du| <= |w| |d x e2| / |det|,
 *   |dv| <= |w| |d x e1| / |det|.
 * The float32 test's own rounding on the perturbed ray is the single-scene
 * bound; first-order terms only, with a factor 2 on the sum for the
 * second-order remainder. */
static void transform_error(const float *m, const float *r, d3 d, const float *tri, double t,
                            double *x_uv, double *x_t)
{
    const double c = 4.0 * 0x1p-24;
    d3 ao, ad;
    double *pao = &ao.x, *pad = &ad.x;
    for (int a = 0; a < 3; ++a) {
        const float *row = m + 4 * a;
        pao[a] = c * (fabs((double)row[0] * r[0]) + fabs((double)row[1] * r[1]) +
                      fabs((double)row[2] * r[2]) + fabs((double)row[3]));
        pad[a] = c * (fabs((double)row[0] * r[4]) + fabs((double)row[1] * r[5]) +
                      fabs((double)row[2] * r[6]));
    }
    double w = d3_norm(ao) + fabs(t) * d3_norm(ad);
    d3 v0 = d3_load(tri), e1 = d3_sub(d3_load(tri + 3), v0), e2 = d3_sub(d3_load(tri + 6), v0);
    double adet = fabs(d3_dot(d, d3_cross(e1, e2)));
    double cu = d3_norm(d3_cross(d, e2)), cv = d3_norm(d3_cross(d, e1));
    *x_uv = w * (cu > cv ? cu : cv) / adet;
    *x_t = w * d3_norm(d3_cross(e1, e2)) / adet;
}

int orc_brute_instanced(const orc_blas *blas, uint32_t n_blas, const orc_inst *inst,
                        uint32_t n_inst, const float *rays, uint32_t n_rays, int kind,
                        const orc_isect *is, double *t_out, uint32_t *prim_out,
                        uint32_t *inst_out, double *u_out, double *v_out, uint8_t *flags,
                        double *bound_uv, double *bound_t)
{
    if (kind == ORC_ALPHA)
        for (uint32_t b = 0; b < n_blas; ++b)
            if (blas[b].n_tris > 0 && !blas[b].texcoords) return -3;
    for (uint32_t i = 0; i < n_rays; ++i) {
        const float *r = rays + 8 * (size_t)i;
        double tmin = r[3], tmax = r[7];
        double t1 = INFINITY, t2 = INFINITY, u1 = 0, v1 = 0, bt1 = 0, bu1 = 0;
        uint32_t p1 = ORC_MISS, q1 = ORC_MISS;
        uint8_t fl = 0;
        for (int pass = 0; pass < 2; ++pass) {
            double reach = (p1 != ORC_MISS) ? t1 + 1e-6 * fabs(t1) + bt1 : tmax;
            for (uint32_t j = 0; j < n_inst; ++j) {
                const orc_inst *in = inst + j;
                if (in->blas >= n_blas) return -2;
                const orc_blas *b = blas + in->blas;
                /* the alpha mask reads this mesh's texture coordinates */
                orc_isect bis = *is;
                bis.texcoords = b->texcoords;
                const float *m = in->m;
                d3 o = {m[0] * (double)r[0] + m[1] * (double)r[1] + m[2] * (double)r[2] + m[3],
                        m[4] * (double)r[0] + m[5] * (double)r[1] + m[6] * (double)r[2] + m[7],
                        m[8] * (double)r[0] + m[9] * (double)r[1] + m[10] * (double)r[2] + m[11]};
                d3 d = {m[0] * (double)r[4] + m[1] * (double)r[5] + m[2] * (double)r[6],
                        m[4] * (double)r[4] + m[5] * (double)r[5] + m[6] * (double)r[6],
                        m[8] * (double)r[4] + m[9] * (double)r[5] + m[10] * (double)r[6]};
                for (uint32_t k = 0; k < b->n_tris; ++k) {
                    double t, u, v, mg, bu, bt;
                    if (!plane_hit64(o, d, b->verts + 9 * (size_t)k, &t, &u, &v, &mg, &bu, &bt)) continue;
                    /* the object ray is a transformed float32 ray: add the
                     * transform's own rounding, carried through the hit */
                    double xu, xt;
                    transform_error(m, r, d, b->verts + 9 * (size_t)k, t, &xu, &xt);
                    bu += 2.0 * xu;
                    bt += 2.0 * xt;
                    const uint32_t g = b->geom ? b->geom[k] : 0;
                    if (pass == 0) {
                        if (!(mg >= 0.0) || !(t > tmin) || !(t < tmax)) continue;
                        double fm;
                        if (kind == ORC_PROCEDURAL && !checker_accept64(is, u, v, &fm)) continue;
                        if (kind == ORC_ALPHA && !alpha_accept64(&bis, k, g, u, v)) continue;
                        if (t < t1) { t2 = t1; t1 = t; u1 = u; v1 = v; p1 = k; q1 = j; bt1 = bt; bu1 = bu; }
                        else if (t < t2) t2 = t;
                    } else {
                        if (!(t > tmin - bt) || !(t < tmax + bt) || !(t <= reach + bt)) continue;
                        double delta = bu > 1e-6 ? bu : 1e-6;
                        if (fabs(mg) < delta) fl |= ORC_E_NEAR_EDGE;
                        if (mg > -delta && kind == ORC_PROCEDURAL) {
                            double fm;
                            checker_accept64(is, u, v, &fm);
                            if (fm < 2.0 * delta * is->checker_n) fl |= ORC_E_NEAR_FILTER;
                        }
                        if (mg > -delta && kind == ORC_ALPHA) {
                            /* as for a single scene: a texel within reach of
                             * the texture coordinates' error deciding otherwise */
                            double wh = is->width > is->height ? is->width : is->height;
                            double reach_tex = (2.0 * delta + 0x1p-20) * wh;
                            if (alpha_decision_fragile(&bis, k, g, u, v, reach_tex))
                                fl |= ORC_E_NEAR_FILTER;
                        }
                        if (p1 != ORC_MISS && !(k == p1 && j == q1) && mg > -delta &&
                            fabs(t - t1) <= bt + bt1)
                            fl |= ORC_E_NEAR_TIE;
                    }
                }
            }
            if (pass == 0 && p1 != ORC_MISS && t2 - t1 < 1e-6 * fabs(t1)) fl |= ORC_E_NEAR_TIE;
        }
        t_out[i] = t1; u_out[i] = u1; v_out[i] = v1; prim_out[i] = p1; inst_out[i] = q1;
        flags[i] = fl;
        if (bound_uv) bound_uv[i] = bu1;
        if (bound_t) bound_t[i] = bt1;
    }
    return 0;
}

/* float32 two-level traversal. */
typedef struct {
    const orc_blas *blas;
    uint32_t n_blas;
    const orc_inst *inst;
    uint32_t n_inst;
    const orc_node *tnodes;   /* top level, built over the instance boxes */
    const uint32_t *tperm;    /* top-level leaf order -> instance index */
    const float *rays;
    uint32_t n_rays;
    int kind;
    orc_isect is;
    int any_hit;
    float *t, *u, *v;
    uint32_t *prim, *inst_id;
    uint32_t *counters;
} inst_job;

static void setup_ray(ray_state *rs, const float o[3], const float d[3])
{
    const float tiny = 0x1p-80f;
    for (int a = 0; a < 3; ++a) {
        rs->o[a] = o[a];
        rs->d[a] = d[a];
        float dd = d[a];
        if (fabsf(dd) < tiny) dd = copysignf(tiny, dd);
        rs->inv[a] = 1.0f / dd;
        rs->ood[a] = o[a] * rs->inv[a];
    }
}

/* One bottom-level traversal with the object ray in rs, on the stack above
 * sp0 (left as found).  Returns 1 iff it accepted a hit. */
static int blas_traverse(const inst_job *job, trav_job *tj, ray_state *rs, uint32_t inst_idx,
                         uint32_t *stack_node, float *stack_tn, int sp0)
{
    const orc_blas *b = job->blas + job->inst[inst_idx].blas;
    if (b->n_tris == 0) return 0;
    tj->verts = b->verts;
    tj->perm = b->perm;
    tj->nodes = b->nodes;
    tj->geom = b->geom;
    tj->is.texcoords = b->texcoords;
    float tn;
    int sp = sp0;
    uint32_t cur = 0;
    int alive = box_test(rs, b->nodes[0].lo, b->nodes[0].hi, &tn);
    const uint32_t acc_before = rs->n_acc;
    while (alive && !rs->done) {
        while (b->nodes[cur].count == 0) {
            const orc_node *nd = &b->nodes[cur];
            float tl, tr;
            int hl = box_test(rs, b->nodes[nd->left].lo, b->nodes[nd->left].hi, &tl);
            int hr = box_test(rs, b->nodes[nd->right].lo, b->nodes[nd->right].hi, &tr);
            if (hl && hr) {
                if (tr < tl) { cur = nd->right; stack_node[sp] = nd->left; stack_tn[sp] = tl; }
                else { cur = nd->left; stack_node[sp] = nd->right; stack_tn[sp] = tr; }
                ++sp;
            } else if (hl) {
                cur = nd->left;
            } else if (hr) {
                cur = nd->right;
            } else {
                alive = 0;
                while (sp > sp0) {
                    --sp;
                    if (!(stack_tn[sp] > rs->tmax_cur)) { cur = stack_node[sp]; alive = 1; break; }
                }
                if (!alive) break;
            }
        }
        if (!alive) break;
        const orc_node *lf = &b->nodes[cur];
        for (uint32_t j = lf->first; j < lf->first + lf->count && !rs->done; ++j)
            tri_test(tj, rs, j);
        if (rs->done) break;
        alive = 0;
        while (sp > sp0) {
            --sp;
            if (!(stack_tn[sp] > rs->tmax_cur)) { cur = stack_node[sp]; alive = 1; break; }
        }
    }
    return rs->n_acc != acc_before;
}

static void inst_one(const inst_job *job, uint32_t i)
{
    const float *r = job->rays + (size_t)i * 8;
    ray_state ws;   /* world ray */
    memset(&ws, 0, sizeof ws);
    setup_ray(&ws, r, r + 4);
    ws.tmin = r[3];
    ws.tmax_cur = r[7];
    ws.prim = ORC_MISS;
    ws.t = INFINITY;
    trav_job tj;
    memset(&tj, 0, sizeof tj);
    tj.kind = job->kind;
    tj.is = job->is;
    tj.any_hit = job->any_hit;
    uint32_t inst_hit = ORC_MISS;
    uint32_t stack_node[256];
    float stack_tn[256];
    int sp = 0;
    if (job->n_inst > 0) {
        float tn;
        uint32_t cur = 0;
        int alive = box_test(&ws, job->tnodes[0].lo, job->tnodes[0].hi, &tn);
        while (alive && !ws.done) {
            while (job->tnodes[cur].count == 0) {
                const orc_node *nd = &job->tnodes[cur];
                float tl, tr;
                int hl = box_test(&ws, job->tnodes[nd->left].lo, job->tnodes[nd->left].hi, &tl);
                int hr = box_test(&ws, job->tnodes[nd->right].lo, job->tnodes[nd->right].hi, &tr);
                if (hl && hr) {
                    if (tr < tl) { cur = nd->right; stack_node[sp] = nd->left; stack_tn[sp] = tl; }
                    else { cur = nd->left; stack_node[sp] = nd->right; stack_tn[sp] = tr; }
                    ++sp;
                } else if (hl) {
                    cur = nd->left;
                } else if (hr) {
                    cur = nd->right;
                } else {
                    alive = 0;
                    while (sp > 0) {
                        --sp;
                        if (!(stack_tn[sp] > ws.tmax_cur)) { cur = stack_node[sp]; alive = 1; break; }
                    }
                    if (!alive) break;
                }
            }
            if (!alive) break;
            const orc_node *lf = &job->tnodes[cur];
            for (uint32_t j = lf->first; j < lf->first + lf->count && !ws.done; ++j) {
                uint32_t q = job->tperm[j];
                const float *m = job->inst[q].m;
                float o[3], d[3];
                for (int a = 0; a < 3; ++a) {
                    o[a] = fmaf(m[4 * a + 0], r[0], fmaf(m[4 * a + 1], r[1], fmaf(m[4 * a + 2], r[2], m[4 * a + 3])));
                    d[a] = fmaf(m[4 * a + 0], r[4], fmaf(m[4 * a + 1], r[5], m[4 * a + 2] * r[6]));
                }
                ray_state os = ws;      /* shares the distance bound and record */
                setup_ray(&os, o, d);
                if (blas_traverse(job, &tj, &os, q, stack_node, stack_tn, sp)) inst_hit = q;
                /* carry back what the object ray changed */
                ws.tmax_cur = os.tmax_cur; ws.prim = os.prim; ws.t = os.t; ws.u = os.u; ws.v = os.v;
                ws.done = os.done;
                ws.n_box = os.n_box; ws.n_tri = os.n_tri; ws.n_cand = os.n_cand; ws.n_acc = os.n_acc;
            }
            if (ws.done) break;
            alive = 0;
            while (sp > 0) {
                --sp;
                if (!(stack_tn[sp] > ws.tmax_cur)) { cur = stack_node[sp]; alive = 1; break; }
            }
        }
    }
    if (ws.prim == ORC_MISS) { ws.t = INFINITY; ws.u = 0.0f; ws.v = 0.0f; inst_hit = ORC_MISS; }
    job->t[i] = ws.t; job->u[i] = ws.u; job->v[i] = ws.v;
    job->prim[i] = ws.prim; job->inst_id[i] = inst_hit;
    if (job->counters) {
        uint32_t *c = job->counters + 4 * (size_t)i;
        c[0] = ws.n_box; c[1] = ws.n_tri; c[2] = ws.n_cand; c[3] = ws.n_acc;
    }
}

int orc_traverse_instanced(const orc_blas *blas, uint32_t n_blas, const orc_inst *inst,
                           uint32_t n_inst, const orc_node *tnodes, const uint32_t *tperm,
                           const float *rays, uint32_t n_rays, int kind, const orc_isect *is,
                           int any_hit, float *t, uint32_t *prim, uint32_t *inst_id, float *u,
                           float *v, uint32_t *counters)
{
    if (kind == ORC_ALPHA)
        for (uint32_t b = 0; b < n_blas; ++b)
            if (blas[b].n_tris > 0 && !blas[b].texcoords) return -3;
    for (uint32_t q = 0; q < n_inst; ++q)
        if (inst[q].blas >= n_blas) return -2;
    inst_job job;
    memset(&job, 0, sizeof job);
    job.blas = blas; job.n_blas = n_blas; job.inst = inst; job.n_inst = n_inst;
    job.tnodes = tnodes; job.tperm = tperm; job.rays = rays; job.n_rays = n_rays;
    job.kind = kind;
    if (is) job.is = *is;
    job.any_hit = any_hit;
    job.t = t; job.u = u; job.v = v; job.prim = prim; job.inst_id = inst_id;
    job.counters = counters;
    for (uint32_t i = 0; i < n_rays; ++i) inst_one(&job, i);
    return 0;
}
