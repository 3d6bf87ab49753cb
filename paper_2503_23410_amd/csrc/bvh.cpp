// Host BVH builder: binned SAH over triangle centroids, parallel over the
// top-level subtrees, with a depth bound that keeps the GPU traversal stack
// finite, then collapsed into 4-wide nodes with 8-bit quantised child boxes
// (64 bytes) packed depth-first.  A 4-wide node halves the node steps of a
// ray against the binary tree and quantisation halves the bytes per node,
// which is what the traversal's memory pipeline pays for; the collapse is
// bounded so that the traversal stack still covers every pending sibling.
//
// Boxes are padded outward by a small absolute margin and rounded outward to
// FP32, so the FP32 slab test on the GPU never rejects a box that holds a
// triangle the watertight test would hit; closest-hit results are therefore
// independent of the tree.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <future>
#include <memory>
#include <numeric>
#include <thread>

#include "vafr_internal.h"

namespace vafr {
namespace {

struct Box {
    float lo[3] = {INFINITY, INFINITY, INFINITY};
    float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    void grow(const float* l, const float* h) {
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], l[k]);
            hi[k] = std::max(hi[k], h[k]);
        }
    }
    void grow_pt(const float* p) { grow(p, p); }
    double area() const {
        if (!(hi[0] >= lo[0])) return 0.0;
        const double dx = (double)hi[0] - lo[0], dy = (double)hi[1] - lo[1], dz = (double)hi[2] - lo[2];
        return 2.0 * (dx * dy + dy * dz + dz * dx);
    }
};

struct Prim {
    float lo[3], hi[3], c[3];
};

struct TNode {
    Box box;
    std::unique_ptr<TNode> l, r;
    int64_t first = 0, count = 0;  // leaf range in idx[]
    int h = 0;                     // internal levels below (0 for a leaf)
};

constexpr int kBins = 32;
constexpr int64_t kParallelMin = 1 << 17;

int ceil_log2(int64_t v) {
    int r = 0;
    while (((int64_t)1 << r) < v) ++r;
    return r;
}

struct Builder {
    const Prim* prims;
    int64_t* idx;
    std::atomic<int> threads_left{0};
    std::atomic<int> max_depth{0};
    std::atomic<int64_t> n_leaves{0};
    int depth_limit = kStackLong;   // leaves stay at depth <= depth_limit - 1

    std::unique_ptr<TNode> build(int64_t first, int64_t n, int depth) {
        auto node = std::make_unique<TNode>();
        Box cb;
        for (int64_t q = first; q < first + n; ++q) {
            const Prim& p = prims[idx[q]];
            node->box.grow(p.lo, p.hi);
            cb.grow_pt(p.c);
        }
        int md = max_depth.load();
        while (depth > md && !max_depth.compare_exchange_weak(md, depth)) {}
        auto make_leaf = [&]() {
            node->first = first;
            node->count = n;
            n_leaves.fetch_add(1);
            return std::move(node);
        };
        if (n <= 1) return make_leaf();
        const bool balance = depth + ceil_log2((n + kMaxLeaf - 1) / kMaxLeaf) >= depth_limit - 1;
        int64_t mid = -1;
        if (!balance) {
            // Binned SAH on all three axes: cost = 1 + (A_L n_L + A_R n_R)/A.
            const double A = node->box.area();
            double best = INFINITY;
            int best_ax = -1, best_split = -1;
            for (int ax = 0; ax < 3; ++ax) {
                const float ext = cb.hi[ax] - cb.lo[ax];
                if (!(ext > 0.0f)) continue;
                const float scale = kBins / ext;
                Box bb[kBins];
                int64_t bn[kBins] = {};
                for (int64_t q = first; q < first + n; ++q) {
                    const Prim& p = prims[idx[q]];
                    int b = (int)((p.c[ax] - cb.lo[ax]) * scale);
                    b = std::min(std::max(b, 0), kBins - 1);
                    bb[b].grow(p.lo, p.hi);
                    ++bn[b];
                }
                double rarea[kBins];
                int64_t rcnt[kBins];
                Box acc;
                int64_t cnt = 0;
                for (int b = kBins - 1; b > 0; --b) {
                    acc.grow(bb[b].lo, bb[b].hi);
                    cnt += bn[b];
                    rarea[b] = acc.area();
                    rcnt[b] = cnt;
                }
                acc = Box();
                cnt = 0;
                for (int b = 0; b < kBins - 1; ++b) {
                    acc.grow(bb[b].lo, bb[b].hi);
                    cnt += bn[b];
                    if (cnt == 0 || rcnt[b + 1] == 0) continue;
                    const double c = 1.0 + (acc.area() * cnt + rarea[b + 1] * rcnt[b + 1]) / std::max(A, 1e-30);
                    if (c < best) { best = c; best_ax = ax; best_split = b; }
                }
            }
            if (n <= kMaxLeaf && (best_ax < 0 || (double)n <= best)) return make_leaf();
            if (best_ax >= 0) {
                const float ext = cb.hi[best_ax] - cb.lo[best_ax];
                const float scale = kBins / ext;
                const float lo = cb.lo[best_ax];
                int64_t* p = std::partition(idx + first, idx + first + n, [&](int64_t t) {
                    int b = (int)((prims[t].c[best_ax] - lo) * scale);
                    b = std::min(std::max(b, 0), kBins - 1);
                    return b <= best_split;
                });
                mid = p - (idx + first);
                if (mid == 0 || mid == n) mid = -1;
            }
        }
        if (mid < 0) {
            if (n <= kMaxLeaf) return make_leaf();
            // Object median along the widest centroid axis.
            int ax = 0;
            for (int k = 1; k < 3; ++k)
                if (cb.hi[k] - cb.lo[k] > cb.hi[ax] - cb.lo[ax]) ax = k;
            mid = n / 2;
            std::nth_element(idx + first, idx + first + mid, idx + first + n,
                             [&](int64_t a, int64_t b) { return prims[a].c[ax] < prims[b].c[ax]; });
        }
        if (n >= kParallelMin && threads_left.fetch_sub(1) > 0) {
            auto fut = std::async(std::launch::async, [&, first, mid, depth]() { return build(first, mid, depth + 1); });
            node->r = build(first + mid, n - mid, depth + 1);
            node->l = fut.get();
        } else {
            node->l = build(first, mid, depth + 1);
            node->r = build(first + mid, n - mid, depth + 1);
        }
        node->h = 1 + std::max(node->l->h, node->r->h);
        return node;
    }
};

struct Packer {
    const float* xyz;
    const int32_t* tri;
    const int64_t* idx;
    float pad;
    int budget;          // stack entries per lane
    HostBvh* out;

    static float down(double v) {
        float f = (float)v;
        if ((double)f > v) f = std::nextafter(f, -INFINITY);
        return f;
    }
    static float up(double v) {
        float f = (float)v;
        if ((double)f < v) f = std::nextafter(f, INFINITY);
        return f;
    }

    int32_t leaf_ref(const TNode* n) {
        const int64_t first = (int64_t)(out->tris.size() / 3);
        for (int64_t q = n->first; q < n->first + n->count; ++q) {
            const int64_t t = idx[q];
            float4 v[3];
            for (int c = 0; c < 3; ++c) {
                const float* p = xyz + 3 * (int64_t)tri[3 * t + c];
                v[c] = make_float4(p[0], p[1], p[2], 0.0f);
            }
            int32_t id = (int32_t)t;
            std::memcpy(&v[0].w, &id, 4);
            out->tris.push_back(v[0]);
            out->tris.push_back(v[1]);
            out->tris.push_back(v[2]);
            out->order.push_back(id);
        }
        return ~(int32_t)((first << 3) | (n->count - 1));
    }

    void child_box(const TNode* c, float* lo, float* hi) {
        for (int k = 0; k < 3; ++k) {
            lo[k] = down((double)c->box.lo[k] - pad);
            hi[k] = up((double)c->box.hi[k] + pad);
        }
    }

    // Emits the subtree of binary node n as 4-wide nodes.  Up to four
    // children are gathered by repeatedly opening the internal child of
    // largest surface area.  `used` is the number of stack entries the
    // traversal may hold on arrival (the sum of children - 1 over the
    // ancestors); a node may gather k children only while
    // used + (k - 1) + (the largest binary height among them) <= budget,
    // so that two children always fit further down and no traversal
    // pushes more than `budget` entries.
    int32_t emit(const TNode* n, int used) {
        if (!n->l) return leaf_ref(n);
        const TNode* ch[4] = {n->l.get(), n->r.get(), nullptr, nullptr};
        int k = 2;
        while (k < 4) {
            int best = -1;
            double best_a = -1.0;
            for (int q = 0; q < k; ++q)
                if (ch[q]->l && ch[q]->box.area() > best_a) {
                    best = q;
                    best_a = ch[q]->box.area();
                }
            if (best < 0) break;
            int hmax = std::max(ch[best]->l->h, ch[best]->r->h);
            for (int q = 0; q < k; ++q)
                if (q != best) hmax = std::max(hmax, ch[q]->h);
            if (used + k + hmax > budget) break;
            const TNode* open = ch[best];
            ch[best] = open->l.get();
            ch[k++] = open->r.get();
        }
        const int32_t me = (int32_t)out->nodes.size();
        out->nodes.push_back(BvhNode{});
        const int below = used + k - 1;
        out->max_stack = std::max(out->max_stack, below);
        float lo[4][3], hi[4][3];
        int32_t ref[4] = {kEmptyRef, kEmptyRef, kEmptyRef, kEmptyRef};
        for (int q = 0; q < 4; ++q) {
            for (int a = 0; a < 3; ++a) {   // an empty slot: [+inf, +inf], skipped by its reference
                lo[q][a] = INFINITY;
                hi[q][a] = INFINITY;
            }
            if (q < k) child_box(ch[q], lo[q], hi[q]);
        }
        for (int q = 0; q < k; ++q) ref[q] = emit(ch[q], below);
        BvhNode& b = out->nodes[me];
        float org[3];
        uint32_t code_lo[3] = {0, 0, 0}, code_hi[3] = {0, 0, 0}, biased[3];
        for (int a = 0; a < 3; ++a) {
            float top = -INFINITY;
            org[a] = INFINITY;
            for (int q = 0; q < k; ++q) {
                org[a] = std::min(org[a], lo[q][a]);
                top = std::max(top, hi[q][a]);
            }
            uint8_t ql[4], qh[4];
            biased[a] = quantise_axis(org[a], top, k, lo, hi, a, ql, qh);
            for (int q = 0; q < 4; ++q) {
                // empty slots keep codes 0 / 0; the traversal skips them by reference
                code_lo[a] |= (uint32_t)(q < k ? ql[q] : 0) << (8 * q);
                code_hi[a] |= (uint32_t)(q < k ? qh[q] : 0) << (8 * q);
            }
        }
        // the scales as FP32 values (2^(biased - 127)), ready for the traversal
        const uint32_t sbits[3] = {biased[0] << 23, biased[1] << 23, biased[2] << 23};
        float sz;
        std::memcpy(&sz, &sbits[2], 4);
        b.org = make_float4(org[0], org[1], org[2], sz);
        b.q0 = make_uint4(code_lo[0], code_hi[0], code_lo[1], code_hi[1]);
        b.q1 = make_uint4(code_lo[2], code_hi[2], sbits[0], sbits[1]);
        b.ref = make_int4(ref[0], ref[1], ref[2], ref[3]);
        return me;
    }

    // 8-bit codes of the children's planes on one axis, relative to origin
    // o with the smallest power-of-two scale that spans up to `top`, each
    // moved outward until fmaf(code, scale, o) lies outside the child's
    // padded box.  Returns the scale's biased FP32 exponent.
    static uint32_t quantise_axis(float o, float top, int k, const float lo[4][3], const float hi[4][3], int a,
                                  uint8_t* ql, uint8_t* qh) {
        const double span = (double)top - (double)o;
        int e = -126;
        if (span > 0.0) {
            std::frexp(span / 255.0, &e);   // span / 255 <= 2^e
            e = std::max(e - 1, -126);
            while (std::ldexp(255.0, e) < span) ++e;
        }
        for (;; ++e) {
            const float sc = std::ldexp(1.0f, e);
            bool fits = true;
            for (int q = 0; q < k && fits; ++q) {
                double fl = std::floor(((double)lo[q][a] - o) / sc), fh = std::ceil(((double)hi[q][a] - o) / sc);
                int cl = (int)std::min(std::max(fl, 0.0), 255.0), ch = (int)std::min(std::max(fh, 0.0), 255.0);
                while (cl > 0 && std::fma((float)cl, sc, o) > lo[q][a]) --cl;
                while (ch < 255 && std::fma((float)ch, sc, o) < hi[q][a]) ++ch;
                if (std::fma((float)cl, sc, o) > lo[q][a] || std::fma((float)ch, sc, o) < hi[q][a]) fits = false;
                ql[q] = (uint8_t)cl;
                qh[q] = (uint8_t)ch;
            }
            if (fits) return (uint32_t)(e + 127);
        }
    }
};

}  // namespace

// Levels of 4-wide nodes on the longest root-to-leaf path.
int wide_depth(const std::vector<BvhNode>& nodes, int32_t root) {
    if (root < 0) return 0;
    std::vector<std::pair<int32_t, int>> todo{{root, 1}};
    int best = 0;
    while (!todo.empty()) {
        const auto [n, d] = todo.back();
        todo.pop_back();
        best = std::max(best, d);
        const int4 r = nodes[n].ref;
        for (int32_t c : {r.x, r.y, r.z, r.w})
            if (c >= 0) todo.push_back({c, d + 1});
    }
    return best;
}

int build_bvh(const float* xyz, int64_t n_verts, const int32_t* tri, int64_t n_tris, HostBvh* out) {
    *out = HostBvh();
    if (n_tris == 0) return VAFR_OK;
    std::vector<Prim> prims(n_tris);
    float ext = 0.0f;
    for (int64_t t = 0; t < n_tris; ++t) {
        Prim& p = prims[t];
        for (int k = 0; k < 3; ++k) { p.lo[k] = INFINITY; p.hi[k] = -INFINITY; }
        for (int c = 0; c < 3; ++c) {
            const int64_t v = tri[3 * t + c];
            if (v < 0 || v >= n_verts) return fail(VAFR_E_ARG, "triangle %lld references vertex %lld of %lld",
                                                   (long long)t, (long long)v, (long long)n_verts);
            for (int k = 0; k < 3; ++k) {
                const float f = xyz[3 * v + k];
                if (!std::isfinite(f)) return fail(VAFR_E_ARG, "vertex %lld is not finite", (long long)v);
                p.lo[k] = std::min(p.lo[k], f);
                p.hi[k] = std::max(p.hi[k], f);
                ext = std::max(ext, std::fabs(f));
            }
        }
        for (int k = 0; k < 3; ++k) p.c[k] = 0.5f * (p.lo[k] + p.hi[k]);
    }
    // node scales stay at most 2^20, so code x scale / d never overflows
    if (ext > 1.0e8f) return fail(VAFR_E_UNSUPPORTED, "scene coordinates beyond 1e8 are not supported");
    std::vector<int64_t> idx(n_tris);
    std::iota(idx.begin(), idx.end(), 0);
    Builder b;
    b.prims = prims.data();
    b.idx = idx.data();
    b.threads_left = (int)std::max(1u, std::thread::hardware_concurrency()) * 2;
    out->stack = ceil_log2((n_tris + kMaxLeaf - 1) / kMaxLeaf) <= kShortStackLevels ? kStackShort : kStackLong;
    b.depth_limit = out->stack;
    std::unique_ptr<TNode> root = b.build(0, n_tris, 0);
    out->max_depth = b.max_depth.load();
    out->n_leaves = b.n_leaves.load();
    out->pad = 2e-5f * (1.0f + ext);
    // fma(plane, 1/d, -o/d) moves a plane by at most 2^-24 |o|: keep that
    // below pad / 8, and |o| small enough that o/d stays finite for the
    // smallest substitute |d| of the traversal (1e-30).
    // The quantised slab test forms fma(code, scale / d, (origin - o) / d);
    // against the decoded plane its distance is that of a plane moved by at
    // most 2^-24 (|o| + |origin - o| + |plane - o|) per axis, below pad / 8
    // while every |o| component stays under pad 2^19 - ext.
    out->fma_origin_limit = std::max(0.0f, std::min(out->pad * 524288.0f - ext, 1.0e7f));
    Packer pk{xyz, tri, idx.data(), out->pad, out->stack + kStackSpill, out};
    out->nodes.reserve(out->n_leaves / 2 + 1);
    out->tris.reserve(3 * n_tris);
    out->order.reserve(n_tris);
    out->root = pk.emit(root.get(), 0);
    out->wide_depth = wide_depth(out->nodes, out->root);
    return VAFR_OK;
}

}  // namespace vafr
