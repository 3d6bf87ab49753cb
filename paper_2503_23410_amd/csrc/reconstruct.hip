// Inverse mapping of an LP buffer onto the display (Sec. 3.2.3,
// Eqs. (10)-(11)).
//
// A workgroup of 4 waves covers a tile of 64 x 4P display pixels; each wave
// writes P rows of 64 consecutive pixels, so the 16-byte RGBA stores of a
// wave form one contiguous 1 KiB segment per row; they are non-temporal
// because the image is written once and not read back here.
//
// VaFR tiles stage their LP texels in LDS first.  Wave 0 bounds the tile's
// footprint in the LP buffer -- the columns between the smallest and the
// largest film radius of the tile and, in each column, the rows between the
// smallest and the largest polar angle, with one texel of margin -- and the
// workgroup copies those texels with row-contiguous loads; the four texels
// of each pixel are then read from LDS.  A texel outside the staged region
// (not expected, but the bound is computed in floating point) is read from
// the LP buffer instead, so the result never depends on the bound.  Tiles
// whose footprint exceeds the LDS budget -- those within a few degrees of
// the gaze point, where one display pixel maps to about one texel or the
// tile surrounds the gaze -- read every texel from the LP buffer.
//
// A view may carry a second LP buffer and image with the same layout, gaze
// and display (the other eye of a binocular frame): every pixel then reads
// the same four texel positions with the same weights in both buffers, so
// the tile stages both (half of the LDS budget each) and maps each pixel
// once for both images.
//
// Tiles are taken in row-major order of the workgroup id, so the eight XCDs
// (which receive consecutive ids in turn) write neighbouring tiles of the
// same tile row at the same time.  Giving each XCD a contiguous band of rows
// instead keeps each XCD's LP reads in its own L2, but makes the stores --
// 97% of the kernel's traffic -- slower: a store-only probe of this pattern
// drops from 6.2 to 5.6 TB/s, and the kernel from 213 to 217 us per
// binocular 8K frame.
#include "vafr_internal.h"

namespace vafr {
namespace {

constexpr int kTileW = 64;
constexpr int kWaves = kReconThreads / 64;
// LDS budget of one tile: staged texels and staged columns (one per lane of
// the wave that builds the column table).
constexpr int kStageTexels = 1024;
constexpr int kStageCols = 64;

// Workgroup id (within one view) -> tile, row-major.
__device__ __forceinline__ void tile_of(int id, int nbx, int& bx, int& by) {
    by = id / nbx;
    bx = id - by * nbx;
}

// Buffer-resource access: 32-bit byte offsets from a uniform base keep the
// per-pixel address arithmetic out of 64-bit VALU operations.  Word 3 of the
// descriptor is the raw-buffer format of gfx9-family GPUs.
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));
constexpr int kRsrcWord3 = 0x00020000;
constexpr int kNonTemporal = 2;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, kRsrcWord3);
}

__device__ __forceinline__ float4 ld4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    const v4u v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), __uint_as_float(v.w));
}

__device__ __forceinline__ v2u ld2(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
}

// Streaming 16-byte store of one pixel.
__device__ __forceinline__ void store_px(__amdgpu_buffer_rsrc_t r, uint32_t off, float4 c) {
    const v4u v = {__float_as_uint(c.x), __float_as_uint(c.y), __float_as_uint(c.z), __float_as_uint(c.w)};
    __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, kNonTemporal);
}

// Polar angle of (dx, dy) in turns, [0, 1], measured from +x toward +y.
// atan on [0, 1] is a degree-15 odd minimax polynomial (coefficients fitted
// for this kernel; FP32 error below 1.4e-7 rad), extended by the octant
// symmetries.
__device__ __forceinline__ float angle_turns(float dx, float dy) {
    const float ax = fabsf(dx), ay = fabsf(dy);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float a = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
    const float z = a * a;
    float p = -0.00405457f;
    p = fmaf(p, z, 0.02186295f);
    p = fmaf(p, z, -0.05591232f);
    p = fmaf(p, z, 0.09642197f);
    p = fmaf(p, z, -0.13908629f);
    p = fmaf(p, z, 0.19946566f);
    p = fmaf(p, z, -0.33329861f);
    p = fmaf(p, z, 0.99999934f);
    float r = p * a * 0.15915494309189535f;                   // [0, 1/8]
    r = ay > ax ? 0.25f - r : r;
    r = dx < 0.0f ? 0.5f - r : r;
    r = dy < 0.0f ? 1.0f - r : r;
    return r;
}

// Rows j0, j1 = j0 + 1 (mod n) and weight t of angular interpolation in a
// column of n rows, for turns in [0, 1]: s = turns n - 0.5 lies in
// [-0.5, n - 0.5], so floor(s) is in [-1, n - 1] and only -1 wraps.
__device__ __forceinline__ void column_rows(int n, float turns, int& j0, int& j1, float& t) {
    const float s = fmaf(turns, (float)n, -0.5f);
    const float fs = floorf(s);
    t = s - fs;
    j0 = (int)fs;
    j0 = j0 < 0 ? j0 + n : j0;
    j1 = j0 + 1 == n ? 0 : j0 + 1;
}

// Weighted sum of four texels.
__device__ __forceinline__ float4 blend4(float4 a, float wa, float4 b, float wb, float4 c, float wc, float4 d,
                                         float wd) {
    return make_float4(fmaf(wd, d.x, fmaf(wc, c.x, fmaf(wb, b.x, wa * a.x))),
                       fmaf(wd, d.y, fmaf(wc, c.y, fmaf(wb, b.y, wa * a.y))),
                       fmaf(wd, d.z, fmaf(wc, c.z, fmaf(wb, b.z, wa * a.z))),
                       fmaf(wd, d.w, fmaf(wc, c.w, fmaf(wb, b.w, wa * a.w))));
}

// Column coordinate a = u(e(rho)) - 0.5 (Eqs. (3), (5), (12)) from the
// FP64-built radial table, already clamped to the first and last column
// centres.
__device__ __forceinline__ float column_coord(const ReconView& v, __amdgpu_buffer_rsrc_t ut, float rho) {
    const float tq = fminf(rho * v.rho_scale, (float)kURhoN);
    const int k = (int)tq;
    const v2u uk = ld2(ut, (uint32_t)k * 8u);
    return fmaf(tq - (float)k, __uint_as_float(uk.y), __uint_as_float(uk.x)) - 0.5f;
}

// One staged column: LP offset and row count of the column, staged rows
// j_start .. j_start + cnt - 1 (mod n) at LDS texels base .. base + cnt - 1.
struct StageCol {
    uint32_t off;
    uint32_t n_cnt;     // n | cnt << 16
    uint32_t js_base;   // j_start | base << 16
};

struct Stage {
    float4 tex[kStageTexels];
    StageCol col[kStageCols];
    int base[kStageCols];   // first LDS texel of each staged column (ascending)
    int i_lo, n_cols;       // staged columns i_lo .. i_lo + n_cols - 1 (n_cols = 0: nothing staged)
    int total;              // staged texels
};

// Where texel j of the column described by (off, n, j_start, cnt, base)
// is: its LDS index when staged (else -1), and its LP byte offset.
struct Tap {
    int lds;
    uint32_t src;
};

__device__ __forceinline__ Tap tap_of(uint32_t off, int n, int js, int cnt, int base, int j) {
    int rel = j - js;
    rel = rel < 0 ? rel + n : rel;
    return Tap{rel < cnt ? base + rel : -1, (off + (uint32_t)j) * 16u};
}

// The texel of tap t in the LP buffer whose staged copy starts at LDS
// texel `half` (0, or kStageTexels / 2 for the second buffer of a pair).
__device__ __forceinline__ float4 texel(const Stage& st, __amdgpu_buffer_rsrc_t lp, int half, const Tap& t) {
    if (t.lds >= 0) return st.tex[half + t.lds];
    return ld4(lp, t.src);
}

// Column i's (offset, rows, staged range): staged columns from LDS, others
// from the column table with an empty staged range.
__device__ __forceinline__ void column_of(const Stage& st, __amdgpu_buffer_rsrc_t ct, int i, uint32_t& off, int& n,
                                          int& js, int& cnt, int& base) {
    const int c = i - st.i_lo;
    if ((unsigned)c < (unsigned)st.n_cols) {
        const StageCol sc = st.col[c];
        off = sc.off;
        n = (int)(sc.n_cnt & 0xffffu);
        cnt = (int)(sc.n_cnt >> 16);
        js = (int)(sc.js_base & 0xffffu);
        base = (int)(sc.js_base >> 16);
    } else {
        const v2u c2 = ld2(ct, (uint32_t)i * 8u);
        n = (int)c2.x;
        off = c2.y;
        js = 0;
        cnt = 0;
        base = 0;
    }
}

// Pixel at film offset (dx, dy) from the gaze point whose column coordinate
// a = u - 0.5 is already known: c from the LP buffer lp and, with kPair, c2
// from the paired buffer lp2 (same positions and weights).
template <bool kPair>
__device__ __forceinline__ void sample_vafr(const ReconView& v, const Stage& st, __amdgpu_buffer_rsrc_t lp,
                                            __amdgpu_buffer_rsrc_t lp2, __amdgpu_buffer_rsrc_t ct, float dx,
                                            float dy, float a, float4& c, float4& c2) {
    int i0 = (int)a;
    i0 = i0 > v.n_cols - 1 ? v.n_cols - 1 : (i0 < 0 ? 0 : i0);
    const int i1 = i0 + 1 < v.n_cols ? i0 + 1 : v.n_cols - 1;
    const float w = a - (float)i0;
    const float turns = angle_turns(dx, dy);
    uint32_t off0, off1;
    int n0, js0, cnt0, base0, n1, js1, cnt1, base1;
    column_of(st, ct, i0, off0, n0, js0, cnt0, base0);
    column_of(st, ct, i1, off1, n1, js1, cnt1, base1);
    int j00, j01, j10, j11;
    float t0, t1;
    column_rows(n0, turns, j00, j01, t0);
    column_rows(n1, turns, j10, j11, t1);
    const Tap ta = tap_of(off0, n0, js0, cnt0, base0, j00), tb = tap_of(off0, n0, js0, cnt0, base0, j01);
    const Tap tc = tap_of(off1, n1, js1, cnt1, base1, j10), td = tap_of(off1, n1, js1, cnt1, base1, j11);
    const float w0 = 1.0f - w;
    const float wa = w0 - w0 * t0, wb = w0 * t0, wc = w - w * t1, wd = w * t1;
    c = blend4(texel(st, lp, 0, ta), wa, texel(st, lp, 0, tb), wb, texel(st, lp, 0, tc), wc, texel(st, lp, 0, td),
               wd);
    if (kPair) {
        constexpr int h = kStageTexels / 2;
        c2 = blend4(texel(st, lp2, h, ta), wa, texel(st, lp2, h, tb), wb, texel(st, lp2, h, tc), wc,
                    texel(st, lp2, h, td), wd);
    }
}

// u / w of the LaFR kernel (Sec. 4.1 Eq. (15)) at log ratio z in [0, 1] of
// a pixel at squared distance r2 (FP64) from the gaze point.
//  - z <= Z_ef: (z (1 - Fa))^(1/Fa).
//  - z > Z_ef: Eq. (15)'s arccos piece, ((2 acos Za - pi) / pi)^(beta/0.7)
//    (1 - U_ef) + U_ef with Za = (1/z - 1/Z_ef) / (1/Z_ef - 1).  Next to the
//    farthest screen corner Za tends to -1, where acos has an unbounded
//    slope, so it is evaluated through eps = 1 + Za = (1 - z) / (z k),
//    k = 1/Z_ef - 1, and acos(eps - 1) = pi - 2 asin(sqrt(eps / 2)):
//    s = 1 - (4 / pi) asin(sqrt(eps / 2)).  1 - z = -ln q / (2 ln L) with
//    q = r2 / R2 and R the farthest corner's distance (ln R = ln L), q formed
//    in FP64: ln q is log1p(q - 1) for q > 1/2, so it keeps its relative
//    precision as r approaches R, and log(q) below (where q - 1 rounded to
//    FP32 would lose the small q's digits).
__device__ __forceinline__ float lafr_u(const ReconView& v, float z, double r2) {
    if (z <= v.lf_zef) return powf(z * v.lf_fa1, v.lf_inv_fa);
    const double q = r2 * v.lf_inv_r2;
    const float lq = q > 0.5 ? log1pf((float)(q - 1.0)) : logf((float)q);
    const float omz = fmaxf(-lq * v.lf_half_inv_lnl, 0.0f);
    const float eps = fminf(omz / ((1.0f - omz) * v.lf_k), 1.0f);
    const float s = fmaf(-4.0f * (float)M_1_PI, asinf(__builtin_amdgcn_sqrtf(0.5f * eps)), 1.0f);
    return (v.lf_bexp == 1.0f ? s : powf(s, v.lf_bexp)) * (1.0f - v.lf_uef) + v.lf_uef;
}

// Pixel (x, y) of an LMFR / LaFR view: the offset from the gaze point is
// formed in FP64 (the gaze is a continuous FP64 position), then rounded.
__device__ __forceinline__ float4 sample_lmfr(const ReconView& v, __amdgpu_buffer_rsrc_t lp, int x, int y) {
    const double dxd = (double)x + v.lm_cx, dyd = (double)y + v.lm_cy;
    const float dx = (float)dxd, dy = (float)dyd;
    const double r2 = dxd * dxd + dyd * dyd;
    const float r = fmaxf(__builtin_amdgcn_sqrtf((float)r2), 1.0f);
    const float z = __log2f(r) * v.inv_L;                     // Eq. (1); inv_L = ln 2 / L
    float u = (v.lf_on ? lafr_u(v, z, r2)                                      // Eq. (15)
                       : v.alpha == 4.0f ? (z * z) * (z * z) : __powf(z, v.alpha)) * (float)v.n_cols;   // Eq. (14)
    u = fminf(fmaxf(u, 0.5f), (float)v.n_cols - 0.5f);
    const float a = u - 0.5f;
    int i0 = (int)a;
    i0 = i0 > v.n_cols - 1 ? v.n_cols - 1 : i0;
    const int i1 = i0 + 1 < v.n_cols ? i0 + 1 : v.n_cols - 1;
    const float w = a - (float)i0;
    int j0, j1;
    float t;
    column_rows(v.lm_h, angle_turns(dx, dy), j0, j1, t);
    const uint32_t o0 = (uint32_t)(i0 * v.lm_h), o1 = (uint32_t)(i1 * v.lm_h);
    const float w0 = 1.0f - w;
    return blend4(ld4(lp, (o0 + j0) * 16u), w0 - w0 * t, ld4(lp, (o0 + j1) * 16u), w0 * t,
                  ld4(lp, (o1 + j0) * 16u), w - w * t, ld4(lp, (o1 + j1) * 16u), w * t);
}

// Wave 0: the staged columns of the tile whose pixel centres span film
// offsets [xl, xh] x [yl, yh] from the gaze point, written to st.col, and
// st.i_lo / st.n_cols (n_cols = 0 when the footprint does not fit).
__device__ void build_stage(const ReconView& v, Stage& st, __amdgpu_buffer_rsrc_t ut, __amdgpu_buffer_rsrc_t ct,
                            float xl, float xh, float yl, float yh, int budget) {
    const int lane = threadIdx.x;
    int n_cols = 0, i_lo = 0, total = 0;
    const bool around_gaze = xl <= 0.0f && xh >= 0.0f && yl <= 0.0f && yh >= 0.0f;
    if (!around_gaze) {
        // radius range: nearest point of the rectangle and farthest corner
        const float qx = fminf(fmaxf(0.0f, xl), xh), qy = fminf(fmaxf(0.0f, yl), yh);
        const float fx = fmaxf(fabsf(xl), fabsf(xh)), fy = fmaxf(fabsf(yl), fabsf(yh));
        const float r_lo = __builtin_amdgcn_sqrtf(fmaf(qx, qx, qy * qy));
        const float r_hi = __builtin_amdgcn_sqrtf(fmaf(fx, fx, fy * fy));
        const int c_lo = (int)column_coord(v, ut, r_lo) - 1;
        const int c_hi = (int)column_coord(v, ut, r_hi) + 2;
        i_lo = c_lo < 0 ? 0 : c_lo;
        const int i_hi = c_hi > v.n_cols - 1 ? v.n_cols - 1 : c_hi;
        n_cols = i_hi - i_lo + 1;
        // angle range: the rectangle does not hold the gaze point, so the
        // extreme angles are those of its corners (taken about the centre
        // direction, which keeps the range unwrapped)
        const float ref = angle_turns(0.5f * (xl + xh), 0.5f * (yl + yh));
        float lo = 0.0f, hi = 0.0f;
        const float cxs[4] = {xl, xh, xl, xh}, cys[4] = {yl, yl, yh, yh};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float d = angle_turns(cxs[k], cys[k]) - ref;
            d = d >= 0.5f ? d - 1.0f : (d < -0.5f ? d + 1.0f : d);
            lo = fminf(lo, d);
            hi = fmaxf(hi, d);
        }
        lo += ref;
        hi += ref;
        if (n_cols > kStageCols) n_cols = 0;
        int cnt = 0, js = 0, n = 0;
        uint32_t off = 0;
        if (lane < n_cols) {
            const v2u c2 = ld2(ct, (uint32_t)(i_lo + lane) * 8u);
            n = (int)c2.x;
            off = c2.y;
            if (n > 0xffff) n_cols = 0;   // the packed column record holds 16-bit row counts
            const int j_lo = (int)floorf(fmaf(lo, (float)n, -0.5f)) - 1;
            const int j_hi = (int)floorf(fmaf(hi, (float)n, -0.5f)) + 2;
            cnt = j_hi - j_lo + 1;
            if (cnt >= n) {
                cnt = n;
                js = 0;
            } else {
                js = j_lo % n;
                js = js < 0 ? js + n : js;
            }
        }
        // exclusive prefix sum of the counts over the wave
        int incl = cnt;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int o = __shfl_up(incl, d, 64);
            if (lane >= d) incl += o;
        }
        total = __shfl(incl, 63, 64);
        if (total > budget || __ballot(n_cols == 0) != 0) n_cols = 0;
        if (n_cols == 0) total = 0;
        if (lane < n_cols) {
            StageCol sc;
            sc.off = off;
            sc.n_cnt = (uint32_t)n | ((uint32_t)cnt << 16);
            sc.js_base = (uint32_t)js | ((uint32_t)(incl - cnt) << 16);
            st.col[lane] = sc;
            st.base[lane] = incl - cnt;
        }
    }
    if (lane == 0) {
        st.i_lo = i_lo;
        st.n_cols = n_cols;
        st.total = total;
    }
}

// Staged texel k: its column (binary search over the column bases) and its
// LP offset.
__device__ __forceinline__ uint32_t stage_source(const Stage& st, int k) {
    int lo = 0, hi = st.n_cols - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (st.base[mid] <= k) lo = mid;
        else hi = mid - 1;
    }
    const StageCol sc = st.col[lo];
    const int n = (int)(sc.n_cnt & 0xffffu), js = (int)(sc.js_base & 0xffffu);
    int j = js + (k - st.base[lo]);
    j = j >= n ? j - n : j;
    return sc.off + (uint32_t)j;
}

// Thread t copies staged texels t, t + 256, ...: all of its loads are issued
// before the first LDS write, so the copy costs one memory latency.  With
// kPair (at most kStageTexels / 2 texels staged) the same texels of lp2 go
// to the upper half.
template <bool kPair>
__device__ __forceinline__ void fill_stage(Stage& st, __amdgpu_buffer_rsrc_t lp, __amdgpu_buffer_rsrc_t lp2) {
    constexpr int kPer = (kPair ? kStageTexels / 2 : kStageTexels) / kReconThreads;
    constexpr int h = kStageTexels / 2;
    const int total = st.total;
    float4 t[kPer], t2[kPair ? kPer : 1];
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
        const int k = threadIdx.x + m * kReconThreads;
        if (k < total) {
            const uint32_t src = stage_source(st, k) * 16u;
            t[m] = ld4(lp, src);
            if (kPair) t2[m] = ld4(lp2, src);
        }
    }
#pragma unroll
    for (int m = 0; m < kPer; ++m) {
        const int k = threadIdx.x + m * kReconThreads;
        if (k < total) {
            st.tex[k] = t[m];
            if (kPair) st.tex[h + k] = t2[m];
        }
    }
}

// Tile `id` of view v: 64 x 4P pixels, P rows per wave.  M is the mapping
// (kModeVafr / kModeLmfr) or -1 to read it from the view.  kPair: a VaFR
// view with a paired buffer (v.lp2, v.img2), written in the same pass.
template <int P, int M, bool kPair = false>
__device__ __forceinline__ void recon_tile(const ReconView& v, int id, Stage& st) {
    constexpr int kTileH = kWaves * P;
    const int nbx = (v.width + kTileW - 1) / kTileW;
    int bx, by;
    tile_of(id, nbx, bx, by);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int x = bx * kTileW + lane;
    const int y0 = by * kTileH;
    const int mode = M >= 0 ? M : v.mode;
    const __amdgpu_buffer_rsrc_t lp = rsrc(v.lp, v.lp_bytes);
    // the tile's rows start at a uniform base; offsets stay 32-bit
    const int rows = v.height - y0 < kTileH ? v.height - y0 : kTileH;
    const __amdgpu_buffer_rsrc_t img = rsrc(v.img + (size_t)y0 * v.width, (uint32_t)(rows * v.width) * 16u);
    if (mode == kModeVafr) {
        const __amdgpu_buffer_rsrc_t ut = rsrc(v.u_of_rho, (kURhoN + 1) * 8);
        const __amdgpu_buffer_rsrc_t ct = rsrc(v.col, (uint32_t)v.n_cols * 8);
        if (wave == 0) {
            const int x_hi = bx * kTileW + kTileW - 1 < v.width - 1 ? bx * kTileW + kTileW - 1 : v.width - 1;
            build_stage(v, st, ut, ct, fmaf((float)(bx * kTileW), v.sx, v.cx), fmaf((float)x_hi, v.sx, v.cx),
                        fmaf((float)y0, v.sy, v.cy), fmaf((float)(y0 + rows - 1), v.sy, v.cy),
                        kPair ? kStageTexels / 2 : kStageTexels);
        }
        const __amdgpu_buffer_rsrc_t lp2 = rsrc(kPair ? v.lp2 : v.lp, v.lp_bytes);
        const __amdgpu_buffer_rsrc_t img2 =
            rsrc((kPair ? v.img2 : v.img) + (size_t)y0 * v.width, (uint32_t)(rows * v.width) * 16u);
        __syncthreads();
        fill_stage<kPair>(st, lp, lp2);
        __syncthreads();
        if (x >= v.width) return;
        const float dx = fmaf((float)x, v.sx, v.cx);
        // the radial table entries of all P pixels are loaded before the
        // first store, so their latencies overlap
        float tq[P];
        v2u uk[P];
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const float dy = fmaf((float)(y0 + wave * P + r), v.sy, v.cy);
            tq[r] = fminf(__builtin_amdgcn_sqrtf(fmaf(dx, dx, dy * dy)) * v.rho_scale, (float)kURhoN);
            uk[r] = ld2(ut, (uint32_t)(int)tq[r] * 8u);
        }
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const int ty = wave * P + r;
            if (ty < rows) {
                const float dy = fmaf((float)(y0 + ty), v.sy, v.cy);
                const float k = (float)(int)tq[r];
                const float a = fmaf(tq[r] - k, __uint_as_float(uk[r].y), __uint_as_float(uk[r].x)) - 0.5f;
                float4 c, c2;
                sample_vafr<kPair>(v, st, lp, lp2, ct, dx, dy, a, c, c2);
                store_px(img, (uint32_t)(ty * v.width + x) * 16u, c);
                if (kPair) store_px(img2, (uint32_t)(ty * v.width + x) * 16u, c2);
            }
        }
    } else {
        if (x >= v.width) return;
        for (int r = 0; r < P; ++r) {
            const int ty = wave * P + r;
            if (ty >= rows) break;
            store_px(img, (uint32_t)(ty * v.width + x) * 16u, sample_lmfr(v, lp, x, y0 + ty));
        }
    }
}

template <int P, int M>
__global__ __launch_bounds__(kReconThreads) void k_recon(const ReconView v) {
    __shared__ Stage st;
    recon_tile<P, M>(v, blockIdx.x, st);
}

// Batched launch over several views (block_end: running tile counts).
template <int P>
__global__ __launch_bounds__(kReconThreads) void k_recon_batch(const ReconView* __restrict__ views,
                                                             const int32_t* __restrict__ block_end, int32_t n_views) {
    __shared__ Stage st;
    const int b = blockIdx.x;
    int vid = 0;
    while (vid + 1 < n_views && b >= block_end[vid]) ++vid;
    const int first = vid ? block_end[vid - 1] : 0;
    const ReconView& v = views[vid];
    if (v.lp2) recon_tile<P, kModeVafr, true>(v, b - first, st);
    else recon_tile<P, -1>(v, b - first, st);
}

}  // namespace

bool recon_rows_ok(int rows) { return rows == 1 || rows == 2 || rows == 4 || rows == 8; }

int64_t recon_blocks_of(const ReconView& v, int rows) {
    const int tile_h = kWaves * rows;
    return (int64_t)((v.width + kTileW - 1) / kTileW) * ((v.height + tile_h - 1) / tile_h);
}

int launch_reconstruct(const ReconView& v, hipStream_t stream, int rows) {
    if (!recon_rows_ok(rows)) return fail(VAFR_E_ARG, "reconstruction rows per thread must be 1, 2, 4 or 8");
    const int64_t blocks = recon_blocks_of(v, rows);
    if (blocks > 0x7fffffff) return fail(VAFR_E_UNSUPPORTED, "display too large");
    const dim3 g((unsigned)blocks), t(kReconThreads);
    if (v.mode == kModeVafr) {
        switch (rows) {
            case 1: hipLaunchKernelGGL((k_recon<1, kModeVafr>), g, t, 0, stream, v); break;
            case 2: hipLaunchKernelGGL((k_recon<2, kModeVafr>), g, t, 0, stream, v); break;
            case 4: hipLaunchKernelGGL((k_recon<4, kModeVafr>), g, t, 0, stream, v); break;
            default: hipLaunchKernelGGL((k_recon<8, kModeVafr>), g, t, 0, stream, v); break;
        }
    } else {
        switch (rows) {
            case 1: hipLaunchKernelGGL((k_recon<1, kModeLmfr>), g, t, 0, stream, v); break;
            case 2: hipLaunchKernelGGL((k_recon<2, kModeLmfr>), g, t, 0, stream, v); break;
            case 4: hipLaunchKernelGGL((k_recon<4, kModeLmfr>), g, t, 0, stream, v); break;
            default: hipLaunchKernelGGL((k_recon<8, kModeLmfr>), g, t, 0, stream, v); break;
        }
    }
    VAFR_HIP(hipGetLastError());
    return VAFR_OK;
}

const void* recon_batch_kernel(int rows) {
    switch (rows) {
        case 1: return reinterpret_cast<const void*>(&k_recon_batch<1>);
        case 2: return reinterpret_cast<const void*>(&k_recon_batch<2>);
        case 4: return reinterpret_cast<const void*>(&k_recon_batch<4>);
        case 8: return reinterpret_cast<const void*>(&k_recon_batch<8>);
        default: return nullptr;
    }
}

int launch_reconstruct_batch(const ReconView* views_dev, const int32_t* block_end_dev, int32_t n_views,
                             int32_t blocks, int rows, hipStream_t stream) {
    if (blocks <= 0) return VAFR_OK;
    if (!recon_rows_ok(rows)) return fail(VAFR_E_ARG, "reconstruction rows per thread must be 1, 2, 4 or 8");
    const dim3 g((unsigned)blocks), t(kReconThreads);
    switch (rows) {
        case 1: hipLaunchKernelGGL(k_recon_batch<1>, g, t, 0, stream, views_dev, block_end_dev, n_views); break;
        case 2: hipLaunchKernelGGL(k_recon_batch<2>, g, t, 0, stream, views_dev, block_end_dev, n_views); break;
        case 4: hipLaunchKernelGGL(k_recon_batch<4>, g, t, 0, stream, views_dev, block_end_dev, n_views); break;
        default: hipLaunchKernelGGL(k_recon_batch<8>, g, t, 0, stream, views_dev, block_end_dev, n_views); break;
    }
    VAFR_HIP(hipGetLastError());
    return VAFR_OK;
}

}  // namespace vafr
