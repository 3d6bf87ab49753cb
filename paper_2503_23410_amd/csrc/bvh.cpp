// Host BVH builder: binned SAH over triangle centroids, parallel over the
// top-level subtrees, with a depth bound that keeps the GPU traversal stack
// finite, then packed depth-first into 64-byte two-wide nodes.
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
        return node;
    }
};

struct Packer {
    const float* xyz;
    const int32_t* tri;
    const int64_t* idx;
    float pad;
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

    int32_t emit(const TNode* n) {
        if (!n->l) return leaf_ref(n);
        const int32_t me = (int32_t)out->nodes.size();
        out->nodes.push_back(BvhNode{});
        float lo0[3], hi0[3], lo1[3], hi1[3];
        child_box(n->l.get(), lo0, hi0);
        child_box(n->r.get(), lo1, hi1);
        const int32_t r0 = emit(n->l.get());
        const int32_t r1 = emit(n->r.get());
        BvhNode& b = out->nodes[me];
        b.a = make_float4(lo0[0], hi0[0], lo0[1], hi0[1]);
        b.b = make_float4(lo1[0], hi1[0], lo1[1], hi1[1]);
        b.c = make_float4(lo0[2], hi0[2], lo1[2], hi1[2]);
        b.d = make_int4(r0, r1, 0, 0);
        return me;
    }
};

}  // namespace

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
    out->fma_origin_limit = std::min(out->pad * 2097152.0f, 1.0e7f);
    Packer pk{xyz, tri, idx.data(), out->pad, out};
    out->nodes.reserve(out->n_leaves);
    out->tris.reserve(3 * n_tris);
    out->order.reserve(n_tris);
    out->root = pk.emit(root.get());
    return VAFR_OK;
}

}  // namespace vafr
