// Host BVH builder of librtx.
//
// The paper traverses a BVH over the scene primitives (Section 3.1) but
// does not describe the construction, so this library fixes one:
//   * triangle box = exact float min/max of its three vertices; centroid =
//     0.5 * (lo + hi) evaluated in double;
//   * a node with <= max_leaf triangles becomes a leaf (max_leaf in 1..7,
//     4 unless the caller chooses otherwise);
//   * otherwise each axis with a non-zero centroid extent is cut into 32
//     equal-width bins, bin = min(31, int((c - cmin) * (32 / extent))); every
//     plane between two bins is costed as area(L) |L| + area(R) |R| (box
//     surface area in double) and the strictly cheapest plane wins, ties going
//     to the lower axis and then the lower plane; the node's triangles are
//     partitioned stably (left keeps its relative order, then right);
//   * with no centroid extent on any axis, or at depth >= 40, the range is
//     split at index count/2 of its current order;
//   * inner nodes are numbered in depth-first preorder, left child first, and
//     the triangle records are written in the final (leaf) order.
//
// Output layout (both little-endian, 16-byte aligned records):
//   inner node, 64 B:  {lo0.x lo0.y lo0.z hi0.x} {hi0.y hi0.z lo1.x lo1.y}
//                      {lo1.z hi1.x hi1.y hi1.z} {ref0 ref1 0 0}
//     child c's box is (loc, hic); refc = (count << 29) | index with count = 0
//     for an inner node (index = its node number) and 1..max_leaf for a leaf (index =
//     its first triangle record).
//   triangle record, 48 B: {v0.xyz, prim_id} {e1.xyz, geom_id} {e2.xyz, 0}
//     with e1 = v1 - v0 and e2 = v2 - v0 rounded to float.
//   compressed inner node, 32 B (compress_nodes): {F.x F.y F.z Q0} {Q1 Q2 ref0 ref1}
//     with frame words F and twelve 8-bit child coordinates Q (see below).
//   packed inner node, 48 B (pack_nodes): the twelve box words of the 64-B
//     node, child c's reference carried in the low bytes of its lo.x, lo.y,
//     lo.z, hi.x words (byte k in the k-th), each moved outward to carry it.
//   four-wide inner node, 128 B (widen_nodes): {lo.x[4]} {hi.x[4]} {lo.y[4]}
//     {hi.y[4]} {lo.z[4]} {hi.z[4]} {ref[4]} {0 0 0 0}, child c in lane c,
//     unused slots (the last ones) with ref 0xFFFFFFFF and a zero box.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <new>
#include <vector>

#include "rt_internal.hpp"

namespace rtx {
namespace {

constexpr int kBins = 32;
constexpr uint32_t kMedianDepth = 40;

struct Box {
    float lo[3], hi[3];
    void clear()
    {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::numeric_limits<float>::infinity();
            hi[a] = -std::numeric_limits<float>::infinity();
        }
    }
    void grow(const Box &b)
    {
        for (int a = 0; a < 3; ++a) {
            lo[a] = b.lo[a] < lo[a] ? b.lo[a] : lo[a];
            hi[a] = b.hi[a] > hi[a] ? b.hi[a] : hi[a];
        }
    }
    double area() const
    {
        const double dx = double(hi[0]) - double(lo[0]);
        const double dy = double(hi[1]) - double(lo[1]);
        const double dz = double(hi[2]) - double(lo[2]);
        return 2.0 * (dx * dy + dy * dz + dz * dx);
    }
};

struct Builder {
    const float *verts;
    std::vector<Box> tbox;
    std::vector<double> cen;   // [n][3]
    std::vector<uint32_t> order, scratch;
    NodeRecord *nodes;
    uint32_t max_leaf = 4;
    uint32_t n_inner = 0;
    uint32_t max_depth = 0;

    struct Split {
        int axis = -1;
        int plane = 0;
        double cmin = 0.0, scale = 0.0;
    };

    static int bin_index(double c, double cmin, double scale)
    {
        int b = int((c - cmin) * scale);
        return b < 0 ? 0 : (b > kBins - 1 ? kBins - 1 : b);
    }

    Box range_box(uint32_t first, uint32_t count) const
    {
        Box b;
        b.clear();
        for (uint32_t i = first; i < first + count; ++i) b.grow(tbox[order[i]]);
        return b;
    }

    Split find_split(uint32_t first, uint32_t count, uint32_t depth) const
    {
        Split best;
        if (depth >= kMedianDepth) return best;
        double cmin[3], cmax[3];
        for (int a = 0; a < 3; ++a) {
            cmin[a] = std::numeric_limits<double>::infinity();
            cmax[a] = -std::numeric_limits<double>::infinity();
        }
        for (uint32_t i = first; i < first + count; ++i) {
            const double *c = &cen[3 * size_t(order[i])];
            for (int a = 0; a < 3; ++a) {
                cmin[a] = c[a] < cmin[a] ? c[a] : cmin[a];
                cmax[a] = c[a] > cmax[a] ? c[a] : cmax[a];
            }
        }
        double best_cost = std::numeric_limits<double>::infinity();
        for (int a = 0; a < 3; ++a) {
            const double ext = cmax[a] - cmin[a];
            if (!(ext > 0.0)) continue;
            const double scale = double(kBins) / ext;
            Box bins[kBins];
            uint32_t cnt[kBins] = {};
            for (auto &b : bins) b.clear();
            for (uint32_t i = first; i < first + count; ++i) {
                const uint32_t k = order[i];
                const int b = bin_index(cen[3 * size_t(k) + a], cmin[a], scale);
                ++cnt[b];
                bins[b].grow(tbox[k]);
            }
            // suffix sweep: right side of every plane
            Box right[kBins];
            uint32_t nright[kBins];
            Box acc;
            acc.clear();
            uint32_t n = 0;
            for (int b = kBins - 1; b >= 1; --b) {
                if (cnt[b]) acc.grow(bins[b]);
                n += cnt[b];
                right[b] = acc;
                nright[b] = n;
            }
            // prefix sweep: left side, cost, strict minimum
            acc.clear();
            n = 0;
            for (int s = 1; s < kBins; ++s) {
                if (cnt[s - 1]) acc.grow(bins[s - 1]);
                n += cnt[s - 1];
                if (n == 0 || nright[s] == 0) continue;
                const double cost = acc.area() * double(n) + right[s].area() * double(nright[s]);
                if (cost < best_cost) {
                    best_cost = cost;
                    best.axis = a;
                    best.plane = s;
                    best.cmin = cmin[a];
                    best.scale = scale;
                }
            }
        }
        return best;
    }

    uint32_t partition(uint32_t first, uint32_t count, const Split &sp)
    {
        if (sp.axis < 0) return count / 2;
        uint32_t w = first, nr = 0;
        for (uint32_t i = first; i < first + count; ++i) {
            const uint32_t k = order[i];
            if (bin_index(cen[3 * size_t(k) + sp.axis], sp.cmin, sp.scale) < sp.plane)
                order[w++] = k;
            else
                scratch[nr++] = k;
        }
        std::memcpy(&order[w], scratch.data(), nr * sizeof(uint32_t));
        return w - first;
    }

    static uint32_t leaf_ref(uint32_t first, uint32_t count) { return (count << 29) | first; }

    static void put_box(NodeRecord &nd, int child, const Box &b)
    {
        float *f = nd.f;
        const int o = child * 6;  // lo0 at 0..2, hi0 at 3..5, lo1 at 6..8, hi1 at 9..11
        f[o + 0] = b.lo[0];
        f[o + 1] = b.lo[1];
        f[o + 2] = b.lo[2];
        f[o + 3] = b.hi[0];
        f[o + 4] = b.hi[1];
        f[o + 5] = b.hi[2];
    }

    // Builds the subtree over order[first, first+count) at `depth`; returns
    // its packed reference.  `box` is the range's bounding box.
    uint32_t build(uint32_t first, uint32_t count, uint32_t depth)
    {
        if (depth > max_depth) max_depth = depth;
        if (count <= max_leaf) return leaf_ref(first, count);
        const uint32_t id = n_inner++;
        const Split sp = find_split(first, count, depth);
        const uint32_t nl = partition(first, count, sp);
        const Box lb = range_box(first, nl);
        const Box rb = range_box(first + nl, count - nl);
        const uint32_t lref = build(first, nl, depth + 1);
        const uint32_t rref = build(first + nl, count - nl, depth + 1);
        NodeRecord &nd = nodes[id];
        std::memset(&nd, 0, sizeof nd);
        put_box(nd, 0, lb);
        put_box(nd, 1, rb);
        nd.u[12] = lref;
        nd.u[13] = rref;
        return id;
    }
};

}  // namespace

uint32_t max_inner_nodes(uint32_t n_tris, uint32_t max_leaf)
{
    return n_tris > max_leaf ? n_tris - 1 : 0;
}

rt_status build_bvh(const float *verts, const uint32_t *geom_ids, uint32_t n_tris,
                    uint32_t max_leaf, NodeRecord *nodes, TriRecord *tris, rt_bvh_info *info)
{
    std::memset(info, 0, sizeof *info);
    info->n_tris = n_tris;
    info->max_leaf = max_leaf;
    if (n_tris == 0) {
        for (int a = 0; a < 3; ++a) {
            info->root_lo[a] = std::numeric_limits<float>::infinity();
            info->root_hi[a] = -std::numeric_limits<float>::infinity();
        }
        return RT_OK;
    }
    try {
        Builder b;
        b.verts = verts;
        b.max_leaf = max_leaf;
        b.tbox.resize(n_tris);
        b.cen.resize(3 * size_t(n_tris));
        b.order.resize(n_tris);
        b.scratch.resize(n_tris);
        b.nodes = nodes;
        for (uint32_t k = 0; k < n_tris; ++k) {
            const float *t = verts + 9 * size_t(k);
            Box &bx = b.tbox[k];
            for (int a = 0; a < 3; ++a) {
                float lo = t[a], hi = t[a];
                lo = t[3 + a] < lo ? t[3 + a] : lo;
                lo = t[6 + a] < lo ? t[6 + a] : lo;
                hi = t[3 + a] > hi ? t[3 + a] : hi;
                hi = t[6 + a] > hi ? t[6 + a] : hi;
                bx.lo[a] = lo;
                bx.hi[a] = hi;
                b.cen[3 * size_t(k) + a] = 0.5 * (double(lo) + double(hi));
            }
            b.order[k] = k;
        }
        const Box root = b.range_box(0, n_tris);
        info->root_ref = b.build(0, n_tris, 0);
        info->n_nodes = b.n_inner;
        info->max_depth = b.max_depth;
        for (int a = 0; a < 3; ++a) {
            info->root_lo[a] = root.lo[a];
            info->root_hi[a] = root.hi[a];
        }
        uint32_t gmax = 0;
        for (uint32_t i = 0; i < n_tris; ++i) {
            const uint32_t k = b.order[i];
            const float *t = verts + 9 * size_t(k);
            TriRecord &r = tris[i];
            r.f[0] = t[0];
            r.f[1] = t[1];
            r.f[2] = t[2];
            r.u[3] = k;
            r.f[4] = t[3] - t[0];
            r.f[5] = t[4] - t[1];
            r.f[6] = t[5] - t[2];
            const uint32_t g = geom_ids ? geom_ids[k] : 0u;
            r.u[7] = g;
            r.f[8] = t[6] - t[0];
            r.f[9] = t[7] - t[1];
            r.f[10] = t[8] - t[2];
            r.u[11] = 0;
            gmax = g > gmax ? g : gmax;
        }
        info->max_geom_id = gmax;
    } catch (const std::bad_alloc &) {
        return RT_ERR_OUT_OF_MEMORY;
    }
    return RT_OK;
}

// -------------------------------------------------------------------------
// 32-byte nodes.  Per axis the frame is the union of the two child boxes
// [L, H]; its origin is the largest float <= L whose pattern has a zero low
// byte, and the low byte holds the exponent E of the scale s = 2^(E - 127),
// the smallest with fma(255, s, origin) >= H.  A coordinate is stored as the
// q in 0..255 whose decoded value fma(q, s, origin) is the tightest one on
// the outside of the exact bound.  decode() is monotone in q and in s (one
// correctly rounded fma of non-negative increments), so each choice is a
// binary search.
// -------------------------------------------------------------------------
namespace {

uint32_t pattern(float f)
{
    uint32_t b;
    std::memcpy(&b, &f, 4);
    return b;
}

float from_pattern(uint32_t b)
{
    float f;
    std::memcpy(&f, &b, 4);
    return f;
}

float frame_origin_of(float lo)
{
    const uint32_t b = pattern(lo);
    if ((b & 0xFFu) == 0) return lo;
    // positive: drop the low byte (smaller value); negative: round the
    // magnitude up to the next pattern with a zero low byte
    return from_pattern((b >> 31) ? (b & ~0xFFu) + 0x100u : (b & ~0xFFu));
}

float decode_q(uint32_t q, float scale, float origin)
{
    return std::fmaf(float(q), scale, origin);
}

}  // namespace

rt_status compress_nodes(const NodeRecord *in, uint32_t n_nodes, NodeQ8Record *out)
{
    for (uint32_t n = 0; n < n_nodes; ++n) {
        const NodeRecord &nd = in[n];
        NodeQ8Record &o = out[n];
        uint8_t q[12];
        for (int a = 0; a < 3; ++a) {
            const float c_lo[2] = {nd.f[a], nd.f[6 + a]};
            const float c_hi[2] = {nd.f[3 + a], nd.f[9 + a]};
            for (int c = 0; c < 2; ++c)
                if (!std::isfinite(c_lo[c]) || !std::isfinite(c_hi[c])) return RT_ERR_INVALID_ARG;
            const float L = c_lo[0] < c_lo[1] ? c_lo[0] : c_lo[1];
            const float H = c_hi[0] > c_hi[1] ? c_hi[0] : c_hi[1];
            const float org = frame_origin_of(L);
            // smallest E in [1, 254] with decode(255) >= H (E = 254 always
            // qualifies: 255 * 2^127 overflows to +inf)
            uint32_t e_lo = 1, e_hi = 254;
            while (e_lo < e_hi) {
                const uint32_t mid = (e_lo + e_hi) / 2;
                if (decode_q(255, from_pattern(mid << 23), org) >= H)
                    e_hi = mid;
                else
                    e_lo = mid + 1;
            }
            const float scale = from_pattern(e_lo << 23);
            o.u[a] = pattern(org) | e_lo;
            for (int c = 0; c < 2; ++c) {
                // largest q with decode(q) <= lo (q = 0 qualifies: origin <= L)
                uint32_t lo_q = 0, hi_q = 255;
                while (lo_q < hi_q) {
                    const uint32_t mid = (lo_q + hi_q + 1) / 2;
                    if (decode_q(mid, scale, org) <= c_lo[c])
                        lo_q = mid;
                    else
                        hi_q = mid - 1;
                }
                q[6 * c + a] = uint8_t(lo_q);
                // smallest q with decode(q) >= hi (q = 255 qualifies)
                lo_q = 0;
                hi_q = 255;
                while (lo_q < hi_q) {
                    const uint32_t mid = (lo_q + hi_q) / 2;
                    if (decode_q(mid, scale, org) >= c_hi[c])
                        hi_q = mid;
                    else
                        lo_q = mid + 1;
                }
                q[6 * c + 3 + a] = uint8_t(lo_q);
            }
        }
        for (int w = 0; w < 3; ++w)
            o.u[3 + w] = uint32_t(q[4 * w]) | uint32_t(q[4 * w + 1]) << 8 |
                         uint32_t(q[4 * w + 2]) << 16 | uint32_t(q[4 * w + 3]) << 24;
        o.u[6] = nd.u[12];
        o.u[7] = nd.u[13];
    }
    return RT_OK;
}

// -------------------------------------------------------------------------
// Refit plan: parents and depths by one preorder sweep (an inner child's
// number is larger than its parent's), subtree sizes by one reverse sweep;
// a node is "top" when its subtree's preorder range leaves its block's.
// -------------------------------------------------------------------------
uint32_t refit_plan(const NodeRecord *nodes, const rt_bvh_info &info, uint32_t *plan)
{
    const uint32_t n = info.n_nodes;
    uint32_t *parent = plan, *depth = plan + n, *top = plan + 2 * size_t(n);
    for (uint32_t k = 0; k < n; ++k) {
        parent[k] = kRefitNoParent;
        depth[k] = 0;
    }
    uint32_t linked = 0;
    for (uint32_t k = 0; k < n; ++k) {
        for (uint32_t c = 0; c < 2; ++c) {
            const uint32_t ref = nodes[k].u[12 + c];
            if ((ref >> 29) != 0) continue;
            const uint32_t ch = ref & kRefIndexMaskHost;
            if (ch <= k || ch >= n || parent[ch] != kRefitNoParent) return UINT32_MAX;
            parent[ch] = 2 * k + c;
            depth[ch] = depth[k] + 1;
            if (depth[ch] > info.max_depth) return UINT32_MAX;  // the kernels sweep 0..max_depth
            ++linked;
        }
    }
    if (n > 0 && linked != n - 1) return UINT32_MAX;  // every node but the root has one parent
    std::vector<uint32_t> size(n, 1);
    for (uint32_t k = n; k-- > 1;) size[parent[k] >> 1] += size[k];
    uint32_t t = 0;
    for (uint32_t k = 0; k < n; ++k) {
        const uint64_t block_end = (uint64_t(k) / kRefitBlockNodes + 1) * kRefitBlockNodes;
        if (uint64_t(k) + size[k] > block_end) {
            depth[k] |= kRefitTopBit;
            top[t++] = k;
        }
    }
    return t;
}

// -------------------------------------------------------------------------
// Packed nodes.  On the key ord(b) = b ^ 0x80000000 (b >= 0) or ~b (b < 0)
// float32 patterns are ordered by value with -0 just below +0, and the low
// byte of a pattern is the key's low byte on the non-negative side and 255
// minus it on the negative side.  Moving a word down to the nearest pattern
// with low byte p steps the key back by the distance between key bytes on
// the word's side; if that crosses below the key of +0, the answer is the
// first key of the negative side with the wanted byte.  Moving up mirrors
// it.  Keys of infinities or NaNs are errors.
// -------------------------------------------------------------------------
namespace {

constexpr uint32_t kZeroKey = 0x80000000u;           // key of +0
constexpr uint32_t kMinFiniteKey = 0x00800000u;      // key of -FLT_MAX
constexpr uint32_t kMaxFiniteKey = 0xFF7FFFFFu;      // key of +FLT_MAX

uint32_t key_of(uint32_t b) { return (b >> 31) ? ~b : b ^ 0x80000000u; }
uint32_t pattern_of_key(uint32_t k) { return k >= kZeroKey ? k ^ 0x80000000u : ~k; }

// The nearest pattern outward from key k (down if lower) whose low byte is
// p, as a key; false if it would leave the finite range.
bool move_key(uint32_t k, uint32_t p, bool lower, uint32_t &out)
{
    if (k < kMinFiniteKey || k > kMaxFiniteKey) return false;
    int64_t r;
    if (lower) {
        if (k >= kZeroKey) {
            r = int64_t(k) - int64_t(((k & 0xFFu) - p) & 0xFFu);
            if (r < int64_t(kZeroKey)) r = int64_t(kZeroKey - 0x100u) | int64_t(0xFFu - p);
        } else {
            r = int64_t(k) - int64_t(((k & 0xFFu) - (0xFFu - p)) & 0xFFu);
        }
        if (r < int64_t(kMinFiniteKey)) return false;
    } else {
        if (k < kZeroKey) {
            r = int64_t(k) + int64_t(((0xFFu - p) - (k & 0xFFu)) & 0xFFu);
            if (r >= int64_t(kZeroKey)) r = int64_t(kZeroKey | p);
        } else {
            r = int64_t(k) + int64_t((p - (k & 0xFFu)) & 0xFFu);
        }
        if (r > int64_t(kMaxFiniteKey)) return false;
    }
    out = uint32_t(r);
    return true;
}

}  // namespace

rt_status pack_nodes(const NodeRecord *in, uint32_t n_nodes, NodePackedRecord *out)
{
    for (uint32_t n = 0; n < n_nodes; ++n) {
        const NodeRecord &nd = in[n];
        NodePackedRecord &o = out[n];
        for (int w = 0; w < 12; ++w) {
            if (!std::isfinite(nd.f[w])) return RT_ERR_INVALID_ARG;
            o.u[w] = nd.u[w];
        }
        for (int c = 0; c < 2; ++c) {
            const uint32_t ref = nd.u[12 + c];
            for (int j = 0; j < 4; ++j) {  // bytes into lo.x, lo.y, lo.z, hi.x
                uint32_t &word = o.u[6 * c + j];
                uint32_t k;
                if (!move_key(key_of(word), (ref >> (8 * j)) & 0xFFu, j < 3, k))
                    return RT_ERR_INVALID_ARG;
                word = pattern_of_key(k);
            }
        }
    }
    return RT_OK;
}

// -------------------------------------------------------------------------
// Four-wide nodes.  A binary node's child list [left, right] grows, while it
// has fewer than four entries and one of them is inner, by replacing the
// inner entry of largest box surface area (double; ties -> the earliest) by
// its two children in place.  The inner entries of the final list are
// collapsed the same way into wide nodes of their own, numbered in
// depth-first preorder; leaf entries keep their binary references.  A wide
// node pushes at most k - 1 stack entries, so the stack bound is the largest
// sum of k - 1 along a root-to-leaf path.
// -------------------------------------------------------------------------
namespace {

struct WideEntry {
    uint32_t ref;
    float lo[3], hi[3];
};

double surface(const WideEntry &e)
{
    const double dx = double(e.hi[0]) - double(e.lo[0]);
    const double dy = double(e.hi[1]) - double(e.lo[1]);
    const double dz = double(e.hi[2]) - double(e.lo[2]);
    return 2.0 * (dx * dy + dy * dz + dz * dx);
}

// The two child slots of binary inner node idx.
void binary_children(const NodeRecord *in, uint32_t idx, WideEntry (&c)[2])
{
    const NodeRecord &nd = in[idx];
    for (int k = 0; k < 2; ++k) {
        for (int a = 0; a < 3; ++a) {
            c[k].lo[a] = nd.f[6 * k + a];
            c[k].hi[a] = nd.f[6 * k + 3 + a];
        }
        c[k].ref = nd.u[12 + k];
    }
}

struct Widener {
    const NodeRecord *in;
    uint32_t n_in;
    NodeW4Record *out;
    uint32_t n_out = 0;

    // Collapses binary inner node idx into wide node n_out; returns the
    // largest sum of k - 1 below and including it, or UINT32_MAX if a child
    // reference is out of range.
    uint32_t collapse(uint32_t idx)
    {
        WideEntry list[4];
        WideEntry two[2];
        binary_children(in, idx, two);
        list[0] = two[0];
        list[1] = two[1];
        uint32_t n = 2;
        while (n < 4) {
            int best = -1;
            double best_area = -1.0;
            for (uint32_t i = 0; i < n; ++i) {
                if ((list[i].ref >> 29) != 0) continue;
                const double a = surface(list[i]);
                if (a > best_area) {
                    best_area = a;
                    best = int(i);
                }
            }
            if (best < 0) break;
            const uint32_t x = list[best].ref & kRefIndexMaskHost;
            if (x >= n_in) return UINT32_MAX;
            binary_children(in, x, two);
            for (uint32_t i = n; i > uint32_t(best) + 1; --i) list[i] = list[i - 1];
            list[best] = two[0];
            list[best + 1] = two[1];
            ++n;
        }
        const uint32_t self = n_out++;
        NodeW4Record &o = out[self];
        std::memset(&o, 0, sizeof o);
        uint32_t deepest = 0;
        for (uint32_t c = 0; c < 4; ++c) {
            if (c >= n) {
                o.u[24 + c] = RT_WIDE_EMPTY_REF;
                continue;
            }
            for (int a = 0; a < 3; ++a) {
                o.f[8 * a + c] = list[c].lo[a];
                o.f[8 * a + 4 + c] = list[c].hi[a];
            }
            uint32_t ref = list[c].ref;
            if ((ref >> 29) == 0) {
                const uint32_t x = ref & kRefIndexMaskHost;
                if (x >= n_in) return UINT32_MAX;
                const uint32_t child = n_out;
                const uint32_t b = collapse(x);
                if (b == UINT32_MAX) return b;
                deepest = b > deepest ? b : deepest;
                ref = child;
            }
            out[self].u[24 + c] = ref;
        }
        return (n - 1) + deepest;
    }
};

}  // namespace

rt_status widen_nodes(const NodeRecord *in, const rt_bvh_info &info, NodeW4Record *out,
                      uint32_t *n_out, uint32_t *stack_bound)
{
    *n_out = 0;
    *stack_bound = 0;
    if ((info.root_ref >> 29) != 0 || info.n_nodes == 0) return RT_OK;  // the root is a leaf
    Widener w{in, info.n_nodes, out};
    const uint32_t root = info.root_ref & kRefIndexMaskHost;
    if (root >= info.n_nodes) return RT_ERR_INVALID_ARG;
    const uint32_t b = w.collapse(root);
    if (b == UINT32_MAX) return RT_ERR_INVALID_ARG;
    *n_out = w.n_out;
    *stack_bound = b;
    return RT_OK;
}

}  // namespace rtx
