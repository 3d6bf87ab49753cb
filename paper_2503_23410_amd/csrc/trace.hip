// Ray generation, BVH traversal, watertight closest hit and shading for the
// LP buffer (Sec. 6.1: one ray per LP texel, closest-hit shading, miss
// shader), the LMFR / LaFR buffers and the full-resolution comparison.
//
// Build with -ffp-contract=off: the ray set-up and the triangle test below
// are written operation by operation so that every rounding is stated, and
// no multiply-add may be fused unless fmaf() says so.
#include "vafr_internal.h"

namespace vafr {
namespace {

// Conservative slab test (Ize, "Robust BVH Ray Traversal", JCGT 2013): the
// exit distance is scaled by 1 + 2 gamma_3 before the overlap test.
constexpr float kExitScale = 1.0000004f;
// Boxes are tested up to the current hit distance scaled by this factor,
// which covers the rounding of a triangle's t relative to its box.
constexpr float kHitSlack = 1.00001f;
constexpr float kTiny = 1e-30f;

// Scene arrays are read through global-address-space pointers: the loads
// become global (not flat) loads, which wait on the vector-memory counter
// only and do not serialise with the LDS stack traffic.
typedef float NFloat4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ldg4(const float4* p, size_t i) {
    const NFloat4 v = ((const __attribute__((address_space(1))) NFloat4*)p)[i];
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint4 ldg_u4(const void* p) {
    const float4 v = ldg4(reinterpret_cast<const float4*>(p), 0);
    return make_uint4(__float_as_uint(v.x), __float_as_uint(v.y), __float_as_uint(v.z), __float_as_uint(v.w));
}
__device__ __forceinline__ int4 ldg_i4(const void* p) {
    const float4 v = ldg4(reinterpret_cast<const float4*>(p), 0);
    return make_int4(__float_as_int(v.x), __float_as_int(v.y), __float_as_int(v.z), __float_as_int(v.w));
}

struct RayPre {
    float ox, oy, oz;
    float dx, dy, dz;
    float ix, iy, iz;       // 1/d with zero components replaced by +-kTiny
    float oix, oiy, oiz;    // o * (1/d), rounded once (slab test in FMA form)
    int kx, ky, kz;
    float Sx, Sy, Sz;
    bool valid;
    bool negx, negy, negz;  // 1/d component negative: the box's high plane is entered first
};

__device__ __forceinline__ float sel3(int k, float a, float b, float c) { return k == 0 ? a : (k == 1 ? b : c); }

__device__ __forceinline__ void ray_setup(float ox, float oy, float oz, float dx, float dy, float dz, RayPre& r) {
    r.ox = ox; r.oy = oy; r.oz = oz;
    r.dx = dx; r.dy = dy; r.dz = dz;
    const float sx = dx == 0.0f ? copysignf(kTiny, dx) : dx;
    const float sy = dy == 0.0f ? copysignf(kTiny, dy) : dy;
    const float sz = dz == 0.0f ? copysignf(kTiny, dz) : dz;
    r.ix = 1.0f / sx;
    r.iy = 1.0f / sy;
    r.iz = 1.0f / sz;
    r.oix = ox * r.ix;
    r.oiy = oy * r.iy;
    r.oiz = oz * r.iz;
    r.negx = r.ix < 0.0f;
    r.negy = r.iy < 0.0f;
    r.negz = r.iz < 0.0f;
    // Watertight set-up: the axis of largest |d| becomes z (first on ties);
    // x, y follow cyclically and swap when d_z < 0.
    int kz = 0;
    float m = fabsf(dx);
    if (fabsf(dy) > m) { kz = 1; m = fabsf(dy); }
    if (fabsf(dz) > m) { kz = 2; }
    int kx = kz == 2 ? 0 : kz + 1;
    int ky = kx == 2 ? 0 : kx + 1;
    const float dkz = sel3(kz, dx, dy, dz);
    if (dkz < 0.0f) { const int t = kx; kx = ky; ky = t; }
    r.kx = kx; r.ky = ky; r.kz = kz;
    r.valid = dkz != 0.0f;
    const float dkx = sel3(kx, dx, dy, dz), dky = sel3(ky, dx, dy, dz);
    r.Sx = dkx / dkz;
    r.Sy = dky / dkz;
    r.Sz = 1.0f / dkz;
}

// Component of (a0, a1, a2) on axis K when K is fixed at compile time, else
// on the lane's axis k.
template <int K>
__device__ __forceinline__ float comp(int k, float a0, float a1, float a2) {
    if constexpr (K == 0) return a0;
    else if constexpr (K == 1) return a1;
    else if constexpr (K == 2) return a2;
    else return sel3(k, a0, a1, a2);
}

// Axis permutation (kx, ky, kz) of the watertight set-up as one number,
// kz * 3 + kx (ky is the remaining axis).
constexpr int perm_code(int kx, int kz) { return kz * 3 + kx; }

// FP32 watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2013).
// Returns true on a hit with t > 0 and writes t = T / det.  KX, KY, KZ fix
// the ray's axis permutation when every lane of the wave shares it, which
// turns the per-lane component selects into plain register choices; -1
// reads it from the ray.  Either way the same operations run on the same
// values.
template <int KX = -1, int KY = -1, int KZ = -1>
__device__ __forceinline__ bool tri_hit(const RayPre& r, float4 v0, float4 v1, float4 v2, float& t_out) {
    const float A0 = v0.x - r.ox, A1 = v0.y - r.oy, A2 = v0.z - r.oz;
    const float B0 = v1.x - r.ox, B1 = v1.y - r.oy, B2 = v1.z - r.oz;
    const float C0 = v2.x - r.ox, C1 = v2.y - r.oy, C2 = v2.z - r.oz;
    const float Akz = comp<KZ>(r.kz, A0, A1, A2), Bkz = comp<KZ>(r.kz, B0, B1, B2);
    const float Ckz = comp<KZ>(r.kz, C0, C1, C2);
    const float Ax = fmaf(-r.Sx, Akz, comp<KX>(r.kx, A0, A1, A2));
    const float Ay = fmaf(-r.Sy, Akz, comp<KY>(r.ky, A0, A1, A2));
    const float Bx = fmaf(-r.Sx, Bkz, comp<KX>(r.kx, B0, B1, B2));
    const float By = fmaf(-r.Sy, Bkz, comp<KY>(r.ky, B0, B1, B2));
    const float Cx = fmaf(-r.Sx, Ckz, comp<KX>(r.kx, C0, C1, C2));
    const float Cy = fmaf(-r.Sy, Ckz, comp<KY>(r.ky, C0, C1, C2));
    // Edge functions with plain products (a shared edge gets exactly
    // negated values in its two triangles).
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    const float det = (U + V) + W;
    if (det == 0.0f || !r.valid) return false;
    const float Az = r.Sz * Akz, Bz = r.Sz * Bkz, Cz = r.Sz * Ckz;
    const float T = (U * Az + V * Bz) + W * Cz;
    const float t = T / det;
    t_out = t;
    return t > 0.0f;
}

// One child box against the ray over [0, tlim] from the distances to its
// entry planes (nx, ny, nz) and exit planes (fx, fy, fz) along each axis:
// tn = entry distance, the return value whether the box is hit.
__device__ __forceinline__ bool slab(float nx, float fx, float ny, float fy, float nz, float fz, float tlim,
                                     float& tn) {
    tn = fmaxf(fmaxf(nx, ny), fmaxf(nz, 0.0f));
    const float tf = fminf(fminf(fx, fy), fminf(fz, tlim));
    return tn <= tf * kExitScale;
}

// Byte c of a code word as a float (the compiler emits one byte-to-float
// conversion for this pattern).
__device__ __forceinline__ float code(uint32_t w, int c) { return (float)((w >> (8 * c)) & 0xffu); }

// Slab distances of a node's quantised child boxes.  Per axis the node
// gives origin g and scale s = 2^k; a plane with code q lies at g + q s.
// Along an axis with 1/d >= 0 the low plane is the entry plane, otherwise
// the high one: the distance is monotone in the code for either form below
// (every rounding is monotone), so choosing the plane words by the sign of
// 1/d gives exactly the min / max of the two distances.
//
// kFma: distance = fma(q, s/d, fma(g, 1/d, -o/d)).  s/d is exact (a power
// of two times 1/d); the inner FMA is the distance to g moved by at most
// 2^-24 |o| (the rounding of o/d) and rounded once; the outer rounds once
// more.  Against the decoded plane this is the exact distance to a plane
// moved by at most 2^-24 (|o| + |g - o| + |plane - o|), well inside the
// padding of every stored box while every |o| component is at most
// TraceView::fma_origin_limit (checked per wave by the caller); relative
// roundings are covered by kExitScale.
//
// Otherwise each plane is decoded as fmaf(q, s, g), which the builder
// checked lies outside the child's padded box, and tested in the
// subtract-multiply form, conservative for any origin.
template <bool kFma>
__device__ __forceinline__ void node_slabs(const RayPre& r, const float4 org, const uint4 q0, const uint4 q1,
                                           float tlim, float tn[4], bool hit[4]) {
    const float sx = __uint_as_float(q1.z), sy = __uint_as_float(q1.w), sz = org.w;
    const uint32_t ex = r.negx ? q0.y : q0.x, xx = r.negx ? q0.x : q0.y;   // entry / exit plane codes
    const uint32_t ey = r.negy ? q0.w : q0.z, xy = r.negy ? q0.z : q0.w;
    const uint32_t ez = r.negz ? q1.y : q1.x, xz = r.negz ? q1.x : q1.y;
    if (kFma) {
        const float bx = fmaf(org.x, r.ix, -r.oix), by = fmaf(org.y, r.iy, -r.oiy), bz = fmaf(org.z, r.iz, -r.oiz);
        const float tx = sx * r.ix, ty = sy * r.iy, tz = sz * r.iz;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            hit[c] = slab(fmaf(code(ex, c), tx, bx), fmaf(code(xx, c), tx, bx), fmaf(code(ey, c), ty, by),
                          fmaf(code(xy, c), ty, by), fmaf(code(ez, c), tz, bz), fmaf(code(xz, c), tz, bz), tlim,
                          tn[c]);
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            hit[c] = slab((fmaf(code(ex, c), sx, org.x) - r.ox) * r.ix, (fmaf(code(xx, c), sx, org.x) - r.ox) * r.ix,
                          (fmaf(code(ey, c), sy, org.y) - r.oy) * r.iy, (fmaf(code(xy, c), sy, org.y) - r.oy) * r.iy,
                          (fmaf(code(ez, c), sz, org.z) - r.oz) * r.iz, (fmaf(code(xz, c), sz, org.z) - r.oz) * r.iz,
                          tlim, tn[c]);
    }
}

// Orders two (distance, reference) pairs.
__device__ __forceinline__ void cswap(float& ka, int& ra, float& kb, int& rb) {
    const bool sw = kb < ka;
    const float k = sw ? kb : ka;
    const int rr = sw ? rb : ra;
    kb = sw ? ka : kb;
    rb = sw ? ra : rb;
    ka = k;
    ra = rr;
}

// Per-lane work counters of the diagnostic pass (node visits, each a test
// of a node's four child boxes; triangle tests).
struct WorkCount {
    uint32_t nodes = 0, tris = 0;
};

// Traversal loop shared by closest-hit and any-hit queries.
//
// Each step of the loop is wave-uniform: either a node step (lanes standing
// on an internal node test its four child boxes, continue with the nearest
// hit child and push the other hit children) or a triangle step (lanes
// holding a parked leaf test its triangles).  A lane parks the first leaf it
// reaches and keeps descending from its stack; the wave switches to the
// triangle step once kParkNum/kParkDen of its live lanes hold a parked leaf,
// or when no lane can take a node step.  This speculative order (Aila and
// Laine, "Understanding the efficiency of ray traversal on GPUs", HPG 2009)
// keeps more of the 64 lanes busy in both steps than descending and testing
// leaves in lock step.  Node steps taken before a parked leaf is tested use
// a hit distance that is not yet the smallest, so they only ever visit more
// boxes; the result is the same (t, id) minimum or the same any-hit bit.
constexpr int kParkNum = 5, kParkDen = 8;

// LDS entries per lane of stack class S (the rest of the stack is scratch).
constexpr int lds_entries(int s) { return s < kStackLds ? s : kStackLds; }

// Triangle step of one lane: the `count` triangles from `first` against the
// ray (axis permutation fixed by KX, KY, KZ, or -1 for the lane's own).
// Closest hit keeps the smallest (t, id) and narrows tlim; any hit stops at
// the first hit (slot_best = 1, ref = kEmptyRef).
template <int KX, int KY, int KZ, bool kAny>
__device__ __forceinline__ void leaf_test(const TraceView& sc, const RayPre& r, int first, int count, float& t_best,
                                          int& id_best, int& slot_best, float& tlim, int& ref) {
    const float4* tp = sc.tris + 3 * (size_t)first;
    for (int q = 0; q < count; ++q) {
        const float4 v0 = ldg4(tp, 3 * q), v1 = ldg4(tp, 3 * q + 1), v2 = ldg4(tp, 3 * q + 2);
        float t;
        if (tri_hit<KX, KY, KZ>(r, v0, v1, v2, t)) {
            if (kAny) {
                slot_best = 1;
                ref = kEmptyRef;
                break;
            }
            const int id = __float_as_int(v0.w);
            if (t < t_best || (t == t_best && id < id_best)) {
                t_best = t;
                id_best = id;
                slot_best = first + q;
                tlim = t * kHitSlack;
            }
        }
    }
}

// Triangle step with the axis permutation fixed when perm names one (a
// wave-uniform value, so the choice is a scalar branch).
template <bool kAny, bool kPerm>
__device__ __forceinline__ void leaf_step(int perm, const TraceView& sc, const RayPre& r, int first, int count,
                                          float& tb, int& ib, int& sb, float& tl, int& ref) {
    if (kPerm) {
        if (perm == perm_code(1, 0)) return leaf_test<1, 2, 0, kAny>(sc, r, first, count, tb, ib, sb, tl, ref);
        if (perm == perm_code(2, 0)) return leaf_test<2, 1, 0, kAny>(sc, r, first, count, tb, ib, sb, tl, ref);
        if (perm == perm_code(2, 1)) return leaf_test<2, 0, 1, kAny>(sc, r, first, count, tb, ib, sb, tl, ref);
        if (perm == perm_code(0, 1)) return leaf_test<0, 2, 1, kAny>(sc, r, first, count, tb, ib, sb, tl, ref);
        if (perm == perm_code(0, 2)) return leaf_test<0, 1, 2, kAny>(sc, r, first, count, tb, ib, sb, tl, ref);
        if (perm == perm_code(1, 2)) return leaf_test<1, 0, 2, kAny>(sc, r, first, count, tb, ib, sb, tl, ref);
    }
    leaf_test<-1, -1, -1, kAny>(sc, r, first, count, tb, ib, sb, tl, ref);
}

// stk points at this lane's column of the block's LDS stack (stride B).
// Closest hit (kAny = false): smallest (t, triangle id); returns the stored
// slot or -1.  Any hit with t > 0 (kAny = true): returns 1 or -1.  With
// kPerm, perm is the rays' axis permutation (perm_code) when every lane of
// the wave shares it, else -1.
template <int B, int S, bool kAny, bool kCount, bool kFma, bool kPerm>
__device__ int traverse_loop(const TraceView& sc, const RayPre& r, int* stk, float& t_best, int& id_best,
                             WorkCount& wc, int perm) {
    t_best = INFINITY;
    id_best = -1;
    // entries 0 .. kLds-1 in the lane's LDS column, the rest in scratch (the
    // two kept in separate branches and address spaces, so that the common
    // case stays an LDS access and the rare one a scratch access, neither a
    // generic one; volatile keeps the spill area in memory instead of in
    // registers)
    constexpr int kLds = lds_entries(S);
    int spill_mem[S + kStackSpill - kLds];
    volatile __attribute__((address_space(5))) int* spill =
        (volatile __attribute__((address_space(5))) int*)spill_mem;
    auto push = [&](int sp_, int v) {
        if (sp_ < kLds) {
            ((__attribute__((address_space(3))) int*)(stk))[sp_ * B] = v;
        } else {
            spill[sp_ - kLds] = v;
        }
    };
    auto top = [&](int sp_) {
        int v;
        if (sp_ < kLds) v = ((__attribute__((address_space(3))) int*)(stk))[sp_ * B];
        else v = spill[sp_ - kLds];
        return v;
    };
    float tlim = INFINITY;   // boxes are tested over [0, t_best * kHitSlack]
    int slot_best = -1;
    int ref = sc.root;   // kEmptyRef: nothing left to visit
    int parked = 0;      // parked leaf reference (< 0); 0 = none
    int sp = 0;
    for (;;) {
        if (ref < 0 && ref != kEmptyRef && parked == 0) {
            parked = ref;
            ref = sp ? top(--sp) : kEmptyRef;
        }
        const uint64_t live = __ballot(ref != kEmptyRef || parked != 0);
        if (live == 0) break;
        const uint64_t at_node = __ballot(ref >= 0);
        const uint64_t holding = __ballot(parked != 0);
        if (at_node != 0 && kParkDen * __popcll(holding) < kParkNum * __popcll(live)) {
            if (ref >= 0) {
                const float4* p = reinterpret_cast<const float4*>(sc.nodes + ref);
                const float4 org = ldg4(p, 0);
                const uint4 q0 = ldg_u4(p + 1), q1 = ldg_u4(p + 2);
                const int4 rf = ldg_i4(p + 3);
                if (kCount) ++wc.nodes;
                float tn[4];
                bool hh[4];
                node_slabs<kFma>(r, org, q0, q1, tlim, tn, hh);
                // empty slots are skipped by their reference
                const bool h0 = hh[0] && rf.x != kEmptyRef, h1 = hh[1] && rf.y != kEmptyRef;
                const bool h2 = hh[2] && rf.z != kEmptyRef, h3 = hh[3] && rf.w != kEmptyRef;
                float k0 = tn[0], k1 = tn[1], k2 = tn[2], k3 = tn[3];
                const int n = (int)h0 + (int)h1 + (int)h2 + (int)h3;
                if (n == 0) {
                    ref = sp ? top(--sp) : kEmptyRef;
                } else if (kAny) {
                    // any hit needs no order: the first hit child next, the
                    // other hit children pushed
                    int nr = kEmptyRef;
                    if (h0) nr = rf.x;
                    if (h1) { if (nr != kEmptyRef) push(sp++, rf.y); else nr = rf.y; }
                    if (h2) { if (nr != kEmptyRef) push(sp++, rf.z); else nr = rf.z; }
                    if (h3) { if (nr != kEmptyRef) push(sp++, rf.w); else nr = rf.w; }
                    ref = nr;
                } else {
                    // nearest hit child next; the others pushed far first
                    k0 = h0 ? k0 : INFINITY;
                    k1 = h1 ? k1 : INFINITY;
                    k2 = h2 ? k2 : INFINITY;
                    k3 = h3 ? k3 : INFINITY;
                    int r0 = rf.x, r1 = rf.y, r2 = rf.z, r3 = rf.w;
                    cswap(k0, r0, k1, r1);
                    cswap(k2, r2, k3, r3);
                    cswap(k0, r0, k2, r2);
                    cswap(k1, r1, k3, r3);
                    cswap(k1, r1, k2, r2);
                    if (n > 3) push(sp++, r3);
                    if (n > 2) push(sp++, r2);
                    if (n > 1) push(sp++, r1);
                    ref = r0;
                }
            }
            continue;
        }
        if (parked != 0) {
            const int x = ~parked;
            parked = 0;
            const int first = x >> 3, count = (x & 7) + 1;
            if (kCount) wc.tris += count;
            leaf_step<kAny, kPerm>(perm, sc, r, first, count, t_best, id_best, slot_best, tlim, ref);
        }
    }
    return slot_best;
}

// The FMA slab test is taken when every lane's origin is within the
// scene's limit (wave-uniform choice, so both loops run without divergence).
// kPerm: the triangle test's axis permutation is fixed for the whole
// traversal when every active lane shares it -- always for shadow rays (one
// light direction), and for most waves of primary rays (a wave covers a
// small screen patch).  The phased path kernels take it for their shadow
// rays only: bounce rays rarely share a permutation, and fixing it for
// every traversal there cost more in registers than it saved.
template <int B, int S, bool kAny, bool kCount, bool kPerm>
__device__ __forceinline__ int traverse(const TraceView& sc, const RayPre& r, int* stk, float& t_best, int& id_best,
                                        WorkCount& wc) {
    const float om = fmaxf(fmaxf(fabsf(r.ox), fabsf(r.oy)), fabsf(r.oz));
    const float oi = fmaxf(fmaxf(fabsf(r.oix), fabsf(r.oiy)), fabsf(r.oiz));
    const bool fma_ok = om <= sc.fma_origin_limit && oi <= 3.0e38f;
    int perm = -1;
    if (kPerm) {
        const int pc = perm_code(r.kx, r.kz);
        const int p0 = __builtin_amdgcn_readfirstlane(pc);
        perm = __ballot(pc != p0) == 0 ? p0 : -1;
    }
    if (__ballot(!fma_ok) == 0)
        return traverse_loop<B, S, kAny, kCount, true, kPerm>(sc, r, stk, t_best, id_best, wc, perm);
    return traverse_loop<B, S, kAny, kCount, false, kPerm>(sc, r, stk, t_best, id_best, wc, perm);
}

template <int B, int S, bool kCount, bool kPerm = false>
__device__ __forceinline__ int closest_hit(const TraceView& sc, const RayPre& r, int* stk, float& t_best,
                                           int& id_best, WorkCount& wc) {
    return traverse<B, S, false, kCount, kPerm>(sc, r, stk, t_best, id_best, wc);
}

template <int B, int S, bool kCount, bool kPerm = false>
__device__ __forceinline__ bool any_hit(const TraceView& sc, const RayPre& r, int* stk, WorkCount& wc) {
    float t;
    int id;
    return traverse<B, S, true, kCount, kPerm>(sc, r, stk, t, id, wc) >= 0;
}

// 32-bit hash of Jarzynski and Olano, "Hash Functions for GPU Rendering",
// JCGT 9(3), 2020 (PCG output permutation of one LCG step).
__device__ __forceinline__ uint32_t pcg_hash(uint32_t v) {
    const uint32_t state = v * 747796405u + 2891336453u;
    const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

__device__ __forceinline__ float3 albedo_of(int id) {
    const uint32_t h = pcg_hash((uint32_t)id);
    return make_float3(0.2f + 0.7f * (float)(h & 255u) / 255.0f, 0.2f + 0.7f * (float)((h >> 8) & 255u) / 255.0f,
                       0.2f + 0.7f * (float)((h >> 16) & 255u) / 255.0f);
}

// Geometric normal facing the ray and the offset origin of the next ray.
__device__ __forceinline__ void hit_frame(const float4 v0, const float4 v1, const float4 v2, const RayPre& r, float t,
                                          float3& n, float3& os) {
    const float e1x = v1.x - v0.x, e1y = v1.y - v0.y, e1z = v1.z - v0.z;
    const float e2x = v2.x - v0.x, e2y = v2.y - v0.y, e2z = v2.z - v0.z;
    float nx = e1y * e2z - e1z * e2y;
    float ny = e1z * e2x - e1x * e2z;
    float nz = e1x * e2y - e1y * e2x;
    const float l2 = (nx * nx + ny * ny) + nz * nz;
    const float len = sqrtf(l2);
    if (len > 0.0f) { nx = nx / len; ny = ny / len; nz = nz / len; }
    const float nd = (nx * r.dx + ny * r.dy) + nz * r.dz;
    if (nd > 0.0f) { nx = -nx; ny = -ny; nz = -nz; }
    const float px = fmaf(t, r.dx, r.ox), py = fmaf(t, r.dy, r.oy), pz = fmaf(t, r.dz, r.oz);
    const float mx = fmaxf(fmaxf(fabsf(px), fabsf(py)), fabsf(pz));
    const float eps = 1e-4f * (1.0f + mx);
    n = make_float3(nx, ny, nz);
    os = make_float3(fmaf(eps, nx, px), fmaf(eps, ny, py), fmaf(eps, nz, pz));
}

__device__ __forceinline__ float rng01(const TraceView& v, uint32_t texel, uint32_t slot) {
    uint32_t h = pcg_hash(v.seed_lo);
    h = pcg_hash(h ^ v.seed_hi);
    h = pcg_hash(h ^ v.frame);
    h = pcg_hash(h ^ v.view);
    h = pcg_hash(h ^ texel);
    h = pcg_hash(h ^ slot);
    return (float)(h >> 8) * (1.0f / 16777216.0f);
}

// Cosine-weighted direction about n: rejection-sampled disk point (up to 8
// tries) lifted to the hemisphere, in the frame of Duff et al. (JCGT 2017).
__device__ __forceinline__ float3 cosine_dir(const TraceView& v, float3 n, uint32_t texel, uint32_t bounce) {
    float x = 0.0f, y = 0.0f;
    for (uint32_t tr = 0; tr < 8; ++tr) {
        const float r0 = rng01(v, texel, bounce * 32u + 2u * tr);
        const float r1 = rng01(v, texel, bounce * 32u + 2u * tr + 1u);
        const float xx = 2.0f * r0 - 1.0f, yy = 2.0f * r1 - 1.0f;
        if (xx * xx + yy * yy < 1.0f) { x = xx; y = yy; break; }
    }
    const float zz = (1.0f - x * x) - y * y;
    const float z = sqrtf(zz > 0.0f ? zz : 0.0f);
    const float s = copysignf(1.0f, n.z);
    const float a = -1.0f / (s + n.z);
    const float b = n.x * n.y * a;
    const float t1x = 1.0f + s * n.x * n.x * a, t1y = s * b, t1z = -s * n.x;
    const float t2x = b, t2y = s + n.y * n.y * a, t2z = -n.y;
    return make_float3((x * t1x + y * t2x) + z * n.x, (x * t1y + y * t2y) + z * n.y, (x * t1z + y * t2z) + z * n.z);
}

// Primary ray direction through film point (Px, Py): (Px R - Py U) + F,
// formed in FP64 operation by operation and rounded to FP32 once.
__device__ __forceinline__ void film_ray(const TraceView& v, double Px, double Py, RayPre& r) {
    float d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double a = Px * (double)v.right[k];
        const double b = Py * (double)v.up[k];
        const double s = a - b;
        d[k] = (float)(s + (double)v.fwd[k]);
    }
    ray_setup(v.eye[0], v.eye[1], v.eye[2], d[0], d[1], d[2], r);
}

// LaFR (Sec. 4.1 Eq. (15)) column -> log ratio z, inverting the kernel piece
// that holds the column's abscissa t = (i + 1/2)/w; FP64 like the LMFR table.
// Out of line and with scalar arguments, so that it adds neither registers
// nor a private copy of the view to the traversal kernels.
__device__ __noinline__ double lafr_column_z(double t, double fa, double uef, double sexp, double zef_inv,
                                             double k) {
    if (t <= uef) return pow(t, fa) / (1.0 - fa);
    const double s = pow((t - uef) / (1.0 - uef), sexp);
    return 1.0 / (zef_inv - sin(0.5 * M_PI * s) * k);
}

// Item -> (ray, output slot).  Returns false for padding items.
__device__ __forceinline__ bool make_item_ray(const TraceView& v, int64_t k, RayPre& r, int64_t& out) {
    if (v.mode == kModeVafr) {
        // trace order: compact screen patches per wave
        const float2 o = v.dxy[k];
        film_ray(v, v.gx + (double)o.x, v.gy + (double)o.y, r);
        out = v.ord[k];
        return true;
    }
    if (v.mode == kModeLmfr) {
        // 8 x 8 tiles of (column, row) of the dense LMFR buffer
        const int tiles_j = (v.lm_h + 7) >> 3;
        const int64_t tile = k >> 6;
        const int w = (int)(k & 63);
        const int64_t i = (tile / tiles_j) * 8 + (w >> 3);
        const int64_t j = (tile % tiles_j) * 8 + (w & 7);
        if (i >= v.lm_w || j >= v.lm_h) return false;
        const double z = v.lf_on ? lafr_column_z(((double)i + 0.5) / (double)v.lm_w, v.lf_fa, v.lf_uef, v.lf_sexp,
                                                 v.lf_zef_inv, v.lf_k)
                                 : v.lm_z[i];
        const double rad = exp(v.lm_L * z);
        const double2 cs = v.lm_cs[j];
        film_ray(v, v.gx + (rad * cs.x) * v.px, v.gy + (rad * cs.y) * v.py, r);
        out = i * v.lm_h + j;
        return true;
    }
    // full resolution, 8 x 8 pixel tiles for coherent waves
    const int tiles_x = (v.width + 7) >> 3;
    const int64_t tile = k >> 6;
    const int w = (int)(k & 63);
    const int x = (int)(tile % tiles_x) * 8 + (w & 7);
    const int y = (int)(tile / tiles_x) * 8 + (w >> 3);
    if (x >= v.width || y >= v.height) return false;
    film_ray(v, ((double)x + 0.5 - 0.5 * (double)v.width) * v.px, ((double)y + 0.5 - 0.5 * (double)v.height) * v.py,
             r);
    out = (int64_t)y * v.width + x;
    return true;
}

template <int B, int S, bool kCount, bool kPerm>
__device__ float4 shade_lambert(const TraceView& v, const RayPre& r, int* stk, int& id_out, WorkCount& wc,
                                uint32_t& n_shadow, float4& p_out) {
    const TraceView& sc = v;
    float t;
    int id;
    const int slot = closest_hit<B, S, kCount, kPerm>(sc, r, stk, t, id, wc);
    id_out = id;
    p_out = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (slot < 0) return make_float4(v.background[0], v.background[1], v.background[2], 1.0f);
    p_out = make_float4(fmaf(t, r.dx, r.ox), fmaf(t, r.dy, r.oy), fmaf(t, r.dz, r.oz), 1.0f);
    const float4* tp = sc.tris + 3 * (size_t)slot;
    float3 n, os;
    hit_frame(ldg4(tp, 0), ldg4(tp, 1), ldg4(tp, 2), r, t, n, os);
    const float ndl = (n.x * v.light_dir[0] + n.y * v.light_dir[1]) + n.z * v.light_dir[2];
    float vis = 1.0f;
    if (ndl > 0.0f && v.shadow) {
        RayPre s;
        ray_setup(os.x, os.y, os.z, v.light_dir[0], v.light_dir[1], v.light_dir[2], s);
        ++n_shadow;
        if (any_hit<B, S, kCount, kPerm>(sc, s, stk, wc)) vis = 0.0f;
    }
    const float lam = ndl > 0.0f ? ndl : 0.0f;
    const float3 a = albedo_of(id);
    return make_float4(a.x * (v.ambient[0] + v.light_rgb[0] * lam * vis),
                       a.y * (v.ambient[1] + v.light_rgb[1] * lam * vis),
                       a.z * (v.ambient[2] + v.light_rgb[2] * lam * vis), 1.0f);
}

// Path from bounce b0 (ray r, throughput thr, radiance L so far): returns
// true when the path has ended (L final), false when it stopped after
// bounce b_last with r set to the next ray.  Bounce 0 reports the primary
// hit id and point.
template <int B, int S, bool kCount>
__device__ bool path_segment(const TraceView& v, RayPre& r, uint32_t texel, int* stk, float3& thr, float3& L,
                             int b0, int b_last, int& id_out, float4& p_out, WorkCount& wc, uint32_t& n_shadow) {
    const TraceView& sc = v;
    for (int bnc = b0; bnc <= v.bounces; ++bnc) {
        float t;
        int id;
        const int slot = closest_hit<B, S, kCount>(sc, r, stk, t, id, wc);
        if (bnc == 0) {
            id_out = id;
            if (slot >= 0) p_out = make_float4(fmaf(t, r.dx, r.ox), fmaf(t, r.dy, r.oy), fmaf(t, r.dz, r.oz), 1.0f);
        }
        if (slot < 0) {
            L.x += thr.x * v.background[0];
            L.y += thr.y * v.background[1];
            L.z += thr.z * v.background[2];
            return true;
        }
        const float4* tp = sc.tris + 3 * (size_t)slot;
        float3 n, os;
        hit_frame(ldg4(tp, 0), ldg4(tp, 1), ldg4(tp, 2), r, t, n, os);
        const float ndl = (n.x * v.light_dir[0] + n.y * v.light_dir[1]) + n.z * v.light_dir[2];
        float vis = 0.0f;
        if (ndl > 0.0f) {
            RayPre s;
            ray_setup(os.x, os.y, os.z, v.light_dir[0], v.light_dir[1], v.light_dir[2], s);
            ++n_shadow;
            vis = any_hit<B, S, kCount>(sc, s, stk, wc) ? 0.0f : 1.0f;
        }
        const float3 a = albedo_of(id);
        thr = make_float3(thr.x * a.x, thr.y * a.y, thr.z * a.z);
        L.x += thr.x * (v.ambient[0] + v.light_rgb[0] * ndl * vis);
        L.y += thr.y * (v.ambient[1] + v.light_rgb[1] * ndl * vis);
        L.z += thr.z * (v.ambient[2] + v.light_rgb[2] * ndl * vis);
        if (bnc == v.bounces) return true;
        const float3 w = cosine_dir(v, n, texel, (uint32_t)bnc);
        ray_setup(os.x, os.y, os.z, w.x, w.y, w.z, r);
        if (bnc == b_last) return false;
    }
    return true;
}

template <int B, int S, bool kCount>
__device__ float4 shade_path(const TraceView& v, RayPre r, uint32_t texel, int* stk, int& id_out, WorkCount& wc,
                             uint32_t& n_shadow, float4& p_out) {
    float3 thr = make_float3(1.0f, 1.0f, 1.0f);
    float3 L = make_float3(0.0f, 0.0f, 0.0f);
    id_out = -1;
    p_out = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    path_segment<B, S, kCount>(v, r, texel, stk, thr, L, 0, 0x7fffffff, id_out, p_out, wc, n_shadow);
    return make_float4(L.x, L.y, L.z, 1.0f);
}

// Compiler-level memory fence: memory written before it is stored before
// it, and memory read after it is loaded again, so that the path state of a
// phased path-mode bounce lives in memory, not in registers, while a
// traversal runs (no instruction is emitted).
__device__ __forceinline__ void state_fence() { __asm__ __volatile__("" ::: "memory"); }

// Bounce `bnc` of a phased path-mode view (batched launches): path p (its
// trace item) with ray r and output index `out`; its throughput and
// radiance so far are (1, 1, 1) and 0 on bounce 0 and come from the path's
// state on later bounces.  The same operations as path_segment, in the
// same order: closest hit; a miss adds thr x background and ends the path;
// a hit multiplies thr by the albedo, and when bounces remain writes the
// next ray (cosine-weighted about the face-forwarded normal, keyed by
// (texel, bnc)) to the path's state and, with `list`, lists p for bounce
// bnc + 1 (one atomic per wave); then the shadow ray toward the light when
// n.l > 0, and L += thr (ambient + light n.l vis), the final radiance on
// the last bounce.  Returns whether the path continues (its next ray is in
// the state).
// Throughput and radiance are read from the state after the closest-hit
// traversal, and throughput, n.l and radiance go through it across the
// shadow ray, so none of them is live during a traversal.  Bounce 0
// reports the primary hit id and point.
template <int B, int S>
__device__ bool path_bounce(const TraceView& v, RayPre& r, int32_t p, int32_t out, int bnc, int* stk, bool list) {
    WorkCount wc;
    float t;
    int id;
    const int slot = closest_hit<B, S, false>(v, r, stk, t, id, wc);
    if (bnc == 0) {
        if (v.out_id) v.out_id[out] = id;
        if (v.out_p)
            v.out_p[out] = slot >= 0 ? make_float4(fmaf(t, r.dx, r.ox), fmaf(t, r.dy, r.oy), fmaf(t, r.dz, r.oz), 1.0f)
                                     : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    float4* st = v.pt_state + 4 * (size_t)p;
    state_fence();
    float3 thr = make_float3(1.0f, 1.0f, 1.0f), L = make_float3(0.0f, 0.0f, 0.0f);
    if (bnc > 0) {
        const float4 th = st[2], lr = st[3];
        thr = make_float3(th.x, th.y, th.z);
        L = make_float3(lr.x, lr.y, lr.z);
    }
    if (slot < 0) {
        L.x += thr.x * v.background[0];
        L.y += thr.y * v.background[1];
        L.z += thr.z * v.background[2];
        v.out_rgba[out] = make_float4(L.x, L.y, L.z, 1.0f);
        return false;
    }
    const float4* tp = v.tris + 3 * (size_t)slot;
    float3 n, os;
    hit_frame(ldg4(tp, 0), ldg4(tp, 1), ldg4(tp, 2), r, t, n, os);
    const float ndl = (n.x * v.light_dir[0] + n.y * v.light_dir[1]) + n.z * v.light_dir[2];
    const float3 a = albedo_of(id);
    thr = make_float3(thr.x * a.x, thr.y * a.y, thr.z * a.z);
    const bool more = bnc < v.bounces;
    if (more) {
        const float3 w = cosine_dir(v, n, (uint32_t)out, (uint32_t)bnc);
        st[0] = make_float4(os.x, os.y, os.z, __int_as_float(out));
        st[1] = make_float4(w.x, w.y, w.z, 0.0f);
        if (list) {
            const uint64_t m = __ballot(1);
            const int lane = (int)__lane_id();
            const int leader = __builtin_ctzll(m);
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(v.pt_count + bnc + 1, (uint32_t)__popcll(m));
            base = __shfl(base, leader, 64);
            v.pt_list[((bnc + 1) & 1) * v.n_items + base + __popcll(m & ((1ull << lane) - 1ull))] = p;
        }
    }
    st[2] = make_float4(thr.x, thr.y, thr.z, ndl);
    st[3] = make_float4(L.x, L.y, L.z, 0.0f);
    float vis = 0.0f;
    state_fence();
    if (ndl > 0.0f) {
        RayPre s;
        ray_setup(os.x, os.y, os.z, v.light_dir[0], v.light_dir[1], v.light_dir[2], s);
        vis = any_hit<B, S, false, true>(v, s, stk, wc) ? 0.0f : 1.0f;
    }
    state_fence();
    const float4 th = st[2], lr = st[3];
    const float4 c = make_float4(lr.x + th.x * (v.ambient[0] + v.light_rgb[0] * th.w * vis),
                                 lr.y + th.y * (v.ambient[1] + v.light_rgb[1] * th.w * vis),
                                 lr.z + th.z * (v.ambient[2] + v.light_rgb[2] * th.w * vis), more ? 0.0f : 1.0f);
    if (more) st[3] = c;
    else v.out_rgba[out] = c;
    return more;
}

// One ray per thread: item `k` of view `v`.  kCount: diagnostic pass that
// counts work into counters[0..3] = primary rays, shadow rays, node visits,
// triangle tests, and writes no image.  kPhased: path-mode views of the
// launch run their bounce 0 as the first phase of path_bounce (batched
// launches only).  kLambert: every view of the launch is Lambert-shaded, so
// the path-tracing code is left out of the kernel.
template <int B, int S, bool kCount, bool kPhased = false, bool kLambert = false>
__device__ __forceinline__ void trace_item(const TraceView& v, int64_t k, int* stack, unsigned long long* counters) {
    RayPre r;
    int64_t out;
    if (k >= v.n_items || !make_item_ray(v, k, r, out)) return;
    int* stk = stack + threadIdx.x;
    if (kPhased && v.pt_phased) {
        // bounces 0 .. kPathFuse by this thread (few paths end before then,
        // and this launch's blocks are XCD-aware and planned); a path still
        // alive after bounce kPathFuse is listed for the queue launches
        const float4* st = v.pt_state + 4 * (size_t)k;
        for (int bnc = 0;; ++bnc) {
            if (!path_bounce<B, S>(v, r, (int32_t)k, (int32_t)out, bnc, stk, bnc >= kPathFuse) || bnc >= kPathFuse)
                break;
            const float4 e0 = st[0], e1 = st[1];
            ray_setup(e0.x, e0.y, e0.z, e1.x, e1.y, e1.z, r);
        }
        return;
    }
    int id;
    float4 c, p;
    WorkCount wc;
    uint32_t n_shadow = 0;
    if (!kLambert && !kPhased && v.shade_mode == VAFR_SHADE_PATH)
        c = shade_path<B, S, kCount>(v, r, (uint32_t)out, stk, id, wc, n_shadow, p);
    else
        c = shade_lambert<B, S, kCount, kLambert>(v, r, stk, id, wc, n_shadow, p);
    if (kCount) {
        atomicAdd(counters + 0, 1ull);
        atomicAdd(counters + 1, (unsigned long long)n_shadow);
        atomicAdd(counters + 2, (unsigned long long)wc.nodes);
        atomicAdd(counters + 3, (unsigned long long)wc.tris);
        return;
    }
    v.out_rgba[out] = c;
    if (v.out_id) v.out_id[out] = id;
    if (v.out_p) v.out_p[out] = p;
}

// Register budget of the traversal kernels, in waves per SIMD (512 VGPRs per
// lane over that many waves, in allocation steps of 8).  Kernels that trace
// whole paths in one pass (per-view path mode, the reprojection's list)
// keep five waves (at most 96 VGPRs): below that their extra state spills.
// The Lambert-only kernels need 63-64 VGPRs (eight waves); their budget of
// six only keeps them from growing.  The phased path-mode kernels hold no
// path state across a traversal and take the eight-wave budget (64 VGPRs)
// without spilling.
#define kTraceWaves(lambert) __attribute__((amdgpu_waves_per_eu((lambert) ? 6 : 5)))
#define kFiveWaves kTraceWaves(false)
#define kBatchWaves(lambert, phased) __attribute__((amdgpu_waves_per_eu((phased) ? 8 : ((lambert) ? 6 : 5))))

// Workgroups are dispatched to the 8 XCDs round-robin.  Work items are
// permuted so that XCD q receives the q-th contiguous eighth of the items:
// rays of one screen region then share their XCD's L2 for the BVH levels
// near the leaves, instead of every L2 holding the whole screen's working
// set.  Workgroup ids past the last multiple of 8 keep their place.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int n) {
    const int per = n / kXcds;
    return b < per * kXcds ? (b % kXcds) * per + b / kXcds : b;
}

// S = stack entries per lane (the scene's stack class).
template <int B, int S, bool kCount, bool kLambert>
__global__ __launch_bounds__(B) kTraceWaves(kLambert) void k_trace(const TraceView v, unsigned long long* counters) {
    __shared__ int stack[lds_entries(S) * B];
    const int b = xcd_block(blockIdx.x, gridDim.x);
    trace_item<B, S, kCount, false, kLambert>(v, (int64_t)b * B + threadIdx.x, stack, counters);
}

// Bounce `bounce` > kPathFuse of the phased path-mode views (batched): workgroup b
// serves view vid with qblock_end[vid-1] <= b < qblock_end[vid]; its thread q
// traces path list[q] of the bounce while q < pt_count[bounce] (workgroups
// past the count exit at once).
template <int S>
__global__ __launch_bounds__(kQueueBlock) kBatchWaves(false, true) void k_trace_queue_batch(
    const TraceView* __restrict__ views, const int32_t* __restrict__ qblock_end, int32_t n_views, int32_t bounce) {
    __shared__ int stack[lds_entries(S) * kQueueBlock];
    const int b = blockIdx.x;
    int vid = 0;
    while (vid + 1 < n_views && b >= qblock_end[vid]) ++vid;
    const TraceView& v = views[vid];
    const int first = vid ? qblock_end[vid - 1] : 0;
    const int64_t q = (int64_t)(b - first) * kQueueBlock + threadIdx.x;
    if (!v.pt_phased || bounce > v.bounces || q >= (int64_t)v.pt_count[bounce]) return;
    const int32_t p = v.pt_list[(bounce & 1) * v.n_items + q];
    const float4* e = v.pt_state + 4 * (size_t)p;
    const float4 e0 = e[0], e1 = e[1];
    RayPre r;
    ray_setup(e0.x, e0.y, e0.z, e1.x, e1.y, e1.z, r);
    path_bounce<kQueueBlock, S>(v, r, p, __float_as_int(e0.w), bounce, stack + threadIdx.x, true);
}

// List mode: thread q < *item_count traces item item_list[q].  The grid is
// sized for the longest list; workgroups past the count exit at once.
// Workgroups keep their hardware order, so a short list still spreads over
// every XCD.
template <int B, int S>
__global__ __launch_bounds__(B) kFiveWaves void k_trace_list(const TraceView v) {
    __shared__ int stack[lds_entries(S) * B];
    const int64_t q = (int64_t)blockIdx.x * B + threadIdx.x;
    if (q >= *v.item_count) return;
    trace_item<B, S, false>(v, v.item_list[q], stack, nullptr);
}

// Batched launch: workgroup b serves view vid with block_end[vid-1] <= b <
// block_end[vid] (block_end is the running sum of per-view workgroups of B
// items each).  S covers the deepest scene of the batch.
// order (nullable): per XCD, the dispatch order of its workgroups'
// blocks (see k_trace_plan); cost (nullable): each block's duration in
// 100 MHz ticks, the larger of its waves', kept for the next frame's plan.
template <int B, int S, bool kCount, bool kPhased, bool kLambert>
__global__ __launch_bounds__(B) kBatchWaves(kLambert, kPhased) void k_trace_batch(const TraceView* __restrict__ views,
                                                   const int32_t* __restrict__ block_end, int32_t n_views,
                                                   unsigned long long* counters, const int32_t* __restrict__ order,
                                                   uint32_t* __restrict__ cost) {
    __shared__ int stack[lds_entries(S) * B];
    const uint64_t t0 = cost ? wall_clock64() : 0;
    int b = xcd_block(blockIdx.x, gridDim.x);
    const int per = gridDim.x / kXcds;
    if (order && (int)blockIdx.x < per * kXcds) {
        const int x = blockIdx.x % kXcds;
        b = x * per + order[x * per + blockIdx.x / kXcds];
    }
    int vid = 0;
    while (vid + 1 < n_views && b >= block_end[vid]) ++vid;
    const int first = vid ? block_end[vid - 1] : 0;
    trace_item<B, S, kCount, kPhased, kLambert>(views[vid], (int64_t)(b - first) * B + threadIdx.x, stack, counters);
    if (cost && (threadIdx.x & 63) == 0) {
        const uint64_t dt = wall_clock64() - t0;
        atomicMax(cost + b, (uint32_t)(dt < 0xffffffffull ? dt : 0xffffffffull));
    }
}

// Longest-first dispatch order of a batched traversal launch, from the
// previous frame's block durations.  Workgroup x plans XCD x, which runs the
// blocks x per .. x per + per - 1 (per = blocks / 8; the few blocks past
// 8 per keep their place): the blocks are ranked into 32 classes of
// duration (two per octave from 2.56 us up, longest first) by a counting
// sort, and order[x per + p] is the p-th block of that ranking, so the
// traversal starts the expensive screen regions first and the cheap ones
// fill in behind them.  Each duration is read once and then cleared for the
// frame being planned; the order is a permutation whatever the durations.
constexpr int kPlanThreads = 1024;
constexpr int kPlanMaxPer = 32768;
constexpr int kPlanClasses = 32;

__global__ __launch_bounds__(kPlanThreads) void k_trace_plan(uint32_t* __restrict__ cost, int32_t* __restrict__ order,
                                                             int32_t blocks) {
    __shared__ uint8_t cls[kPlanMaxPer];
    __shared__ int hist[kPlanClasses], base[kPlanClasses];
    const int per = blocks / kXcds;
    const int x = blockIdx.x;
    const int t = threadIdx.x;
    if (t < kPlanClasses) hist[t] = 0;
    __syncthreads();
    for (int i = t; i < per; i += kPlanThreads) {
        const uint32_t c = cost[x * per + i];
        cost[x * per + i] = 0u;
        // level = 2 log2(c) in half octaves from 2^8 ticks; longer is earlier
        const uint32_t bits = __float_as_uint((float)c);
        int lvl = c ? (int)(bits >> 22) - ((127 + 8) << 1) : 0;
        lvl = lvl < 0 ? 0 : (lvl > kPlanClasses - 1 ? kPlanClasses - 1 : lvl);
        const int k = kPlanClasses - 1 - lvl;
        cls[i] = (uint8_t)k;
        atomicAdd(&hist[k], 1);
    }
    __syncthreads();
    if (t == 0) {
        int acc = 0;
        for (int k = 0; k < kPlanClasses; ++k) {
            base[k] = acc;
            acc += hist[k];
        }
    }
    __syncthreads();
    for (int i = t; i < per; i += kPlanThreads) {
        const int pos = atomicAdd(&base[cls[i]], 1);
        order[x * per + pos] = i;
    }
}

template <int B, int S>
void launch_single(const TraceView& v, int64_t blocks, hipStream_t stream, unsigned long long* counters) {
    if (v.item_list)
        hipLaunchKernelGGL((k_trace_list<B, S>), dim3((unsigned)blocks), dim3(B), 0, stream, v);
    else if (counters)
        hipLaunchKernelGGL((k_trace<B, S, true, false>), dim3((unsigned)blocks), dim3(B), 0, stream, v, counters);
    else if (v.shade_mode == VAFR_SHADE_PATH)
        hipLaunchKernelGGL((k_trace<B, S, false, false>), dim3((unsigned)blocks), dim3(B), 0, stream, v, counters);
    else
        hipLaunchKernelGGL((k_trace<B, S, false, true>), dim3((unsigned)blocks), dim3(B), 0, stream, v, counters);
}

template <int B, int S>
void launch_batch(const TraceView* views, const int32_t* block_end, int32_t n_views, int32_t blocks, bool phased,
                  bool lambert, hipStream_t stream, unsigned long long* counters, const int32_t* order,
                  uint32_t* cost) {
    if (counters)
        hipLaunchKernelGGL((k_trace_batch<B, S, true, false, false>), dim3((unsigned)blocks), dim3(B), 0, stream,
                           views, block_end, n_views, counters, order, cost);
    else if (phased || !lambert)
        hipLaunchKernelGGL((k_trace_batch<B, S, false, true, false>), dim3((unsigned)blocks), dim3(B), 0, stream,
                           views, block_end, n_views, counters, order, cost);
    else
        hipLaunchKernelGGL((k_trace_batch<B, S, false, false, true>), dim3((unsigned)blocks), dim3(B), 0, stream,
                           views, block_end, n_views, counters, order, cost);
}

template <int S>
void launch_single_s(const TraceView& v, int64_t blocks, int block, hipStream_t stream,
                     unsigned long long* counters) {
    if (block == 64) launch_single<64, S>(v, blocks, stream, counters);
    else if (block == 128) launch_single<128, S>(v, blocks, stream, counters);
    else launch_single<256, S>(v, blocks, stream, counters);
}

template <int S>
void launch_batch_s(const TraceView* views, const int32_t* block_end, int32_t n_views, int32_t blocks, int block,
                    bool phased, bool lambert, hipStream_t stream, unsigned long long* counters, const int32_t* order,
                    uint32_t* cost) {
    if (block == 64)
        launch_batch<64, S>(views, block_end, n_views, blocks, phased, lambert, stream, counters, order, cost);
    else if (block == 128)
        launch_batch<128, S>(views, block_end, n_views, blocks, phased, lambert, stream, counters, order, cost);
    else launch_batch<256, S>(views, block_end, n_views, blocks, phased, lambert, stream, counters, order, cost);
}

template <int S, bool kPhased, bool kLambert>
const void* batch_kernel_s(int block) {
    if (block == 64) return reinterpret_cast<const void*>(&k_trace_batch<64, S, false, kPhased, kLambert>);
    if (block == 128) return reinterpret_cast<const void*>(&k_trace_batch<128, S, false, kPhased, kLambert>);
    if (block == 256) return reinterpret_cast<const void*>(&k_trace_batch<256, S, false, kPhased, kLambert>);
    return nullptr;
}

template <int S>
const void* batch_kernel_any(int block, bool phased, bool lambert) {
    if (phased || !lambert) return batch_kernel_s<S, true, false>(block);
    return batch_kernel_s<S, false, true>(block);
}

bool stack_ok(int stack) { return stack == kStackShort || stack == kStackLong; }

}  // namespace

int64_t trace_items_of(const TraceView& v) {
    if (v.mode == kModeFull) return (int64_t)((v.width + 7) / 8) * ((v.height + 7) / 8) * 64;
    if (v.mode == kModeLmfr) return (int64_t)((v.lm_w + 7) / 8) * ((v.lm_h + 7) / 8) * 64;
    return v.n_items;
}

bool trace_block_ok(int block) { return block == 64 || block == 128 || block == 256; }

int launch_trace(const TraceView& v, hipStream_t stream, unsigned long long* counters, int block) {
    if (v.n_items <= 0) return VAFR_OK;
    if (!trace_block_ok(block)) return fail(VAFR_E_ARG, "trace workgroup size must be 64, 128 or 256");
    if (!stack_ok(v.stack)) return fail(VAFR_E_ARG, "unknown traversal stack class %d", v.stack);
    const int64_t blocks = (v.n_items + block - 1) / block;
    if (v.item_list && counters) return fail(VAFR_E_UNSUPPORTED, "work counting does not take an item list");
    if (blocks > 0x7fffffff) return fail(VAFR_E_UNSUPPORTED, "too many rays in one launch");
    if (v.stack == kStackShort) launch_single_s<kStackShort>(v, blocks, block, stream, counters);
    else launch_single_s<kStackLong>(v, blocks, block, stream, counters);
    VAFR_HIP(hipGetLastError());
    return VAFR_OK;
}

const void* trace_batch_kernel(int block, int stack, bool phased, bool lambert) {
    if (stack == kStackShort) return batch_kernel_any<kStackShort>(block, phased, lambert);
    if (stack == kStackLong) return batch_kernel_any<kStackLong>(block, phased, lambert);
    return nullptr;
}

int launch_trace_batch(const TraceView* views_dev, const int32_t* block_end_dev, int32_t n_views, int32_t blocks,
                       int block, int stack, bool phased, bool lambert, hipStream_t stream,
                       unsigned long long* counters, const int32_t* order, uint32_t* cost) {
    if (blocks <= 0) return VAFR_OK;
    if (!trace_block_ok(block)) return fail(VAFR_E_ARG, "trace workgroup size must be 64, 128 or 256");
    if (!stack_ok(stack)) return fail(VAFR_E_ARG, "unknown traversal stack class %d", stack);
    if (order && !trace_plan_ok(blocks)) return fail(VAFR_E_ARG, "too many blocks for a planned launch");
    if (stack == kStackShort)
        launch_batch_s<kStackShort>(views_dev, block_end_dev, n_views, blocks, block, phased, lambert, stream,
                                    counters, order, cost);
    else
        launch_batch_s<kStackLong>(views_dev, block_end_dev, n_views, blocks, block, phased, lambert, stream,
                                   counters, order, cost);
    VAFR_HIP(hipGetLastError());
    return VAFR_OK;
}

bool trace_plan_ok(int32_t blocks) { return blocks / kXcds <= kPlanMaxPer; }

const void* trace_queue_batch_kernel(int stack) {
    if (stack == kStackShort) return reinterpret_cast<const void*>(&k_trace_queue_batch<kStackShort>);
    if (stack == kStackLong) return reinterpret_cast<const void*>(&k_trace_queue_batch<kStackLong>);
    return nullptr;
}

int launch_trace_queue_batch(const TraceView* views_dev, const int32_t* qblock_end_dev, int32_t n_views,
                             int32_t blocks, int stack, int bounce, hipStream_t stream) {
    if (blocks <= 0) return VAFR_OK;
    if (!stack_ok(stack)) return fail(VAFR_E_ARG, "unknown traversal stack class %d", stack);
    if (bounce < 1 || bounce > kMaxBounces) return fail(VAFR_E_ARG, "bounce %d out of range", bounce);
    if (stack == kStackShort)
        hipLaunchKernelGGL((k_trace_queue_batch<kStackShort>), dim3((unsigned)blocks), dim3(kQueueBlock), 0, stream,
                           views_dev, qblock_end_dev, n_views, (int32_t)bounce);
    else
        hipLaunchKernelGGL((k_trace_queue_batch<kStackLong>), dim3((unsigned)blocks), dim3(kQueueBlock), 0, stream,
                           views_dev, qblock_end_dev, n_views, (int32_t)bounce);
    VAFR_HIP(hipGetLastError());
    return VAFR_OK;
}

const void* trace_plan_kernel() { return reinterpret_cast<const void*>(&k_trace_plan); }

int launch_trace_plan(uint32_t* cost, int32_t* order, int32_t blocks, hipStream_t stream) {
    if (blocks <= 0) return VAFR_OK;
    if (!trace_plan_ok(blocks)) return fail(VAFR_E_ARG, "too many blocks for a planned launch");
    hipLaunchKernelGGL(k_trace_plan, dim3(kXcds), dim3(kPlanThreads), 0, stream, cost, order, blocks);
    VAFR_HIP(hipGetLastError());
    return VAFR_OK;
}

}  // namespace vafr
