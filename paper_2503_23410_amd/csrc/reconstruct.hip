// Inverse mapping of an LP buffer onto the display (Sec. 3.2.3,
// Eqs. (10)-(11)), one thread per display pixel.
//
// A workgroup covers a tile of 64 x R display pixels; each wave covers 64
// consecutive pixels of one row, so the 16-byte RGBA stores of a wave form one
// contiguous 1 KiB segment; they are non-temporal because the image is
// written once and not read back here.  The LP buffer (17 MB per VaFR view)
// is read through the caches: a texel feeds tens of display pixels in the
// periphery.  The kernel is bound by its arithmetic per pixel (measured), so
// the forward map is reduced to one radial table lookup and one polynomial
// angle evaluation.
//
// Workgroups are mapped XCD-aware: consecutive workgroup ids land on
// different XCDs, so ids are permuted such that each XCD receives a
// contiguous band of display rows and reads a compact part of the LP buffer
// through its own L2.
#include "vafr_internal.h"

namespace vafr {
namespace {

constexpr int kTileW = 64;
constexpr int kXcds = 8;

// Workgroup id (within one view) -> tile, so that XCD q (= id mod 8) gets the
// q-th contiguous eighth of the tiles in row-major order.
__device__ __forceinline__ void xcd_tile(int id, int nbx, int nby, int& bx, int& by) {
    const int n = nbx * nby;
    int t = id;
    if (n >= kXcds * 64) {
        const int per = n / kXcds;
        if (id < per * kXcds) t = (id % kXcds) * per + id / kXcds;
    }
    bx = t % nbx;
    by = t / nbx;
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

// Rows j0, j1 and weight t of angular interpolation in a column of n rows.
__device__ __forceinline__ void column_rows(int n, float turns, int& j0, int& j1, float& t) {
    const float s = fmaf(turns, (float)n, -0.5f);
    const float fs = floorf(s);
    t = s - fs;
    j0 = (int)fs;
    j0 = j0 < 0 ? j0 + n : (j0 >= n ? j0 - n : j0);
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

__device__ __forceinline__ float4 sample_vafr(const ReconView& v, float dx, float dy) {
    const __amdgpu_buffer_rsrc_t lp = rsrc(v.lp, v.lp_bytes);
    const __amdgpu_buffer_rsrc_t ut = rsrc(v.u_of_rho, (kURhoN + 1) * 8);
    const __amdgpu_buffer_rsrc_t ct = rsrc(v.col, (uint32_t)v.n_cols * 8);
    const float rho = __builtin_amdgcn_sqrtf(fmaf(dx, dx, dy * dy));
    // u(e(rho)) (Eqs. (3), (5), (12)) from the FP64-built radial table,
    // already clamped to the first and last column centres.
    const float tq = fminf(rho * v.rho_scale, (float)kURhoN);
    const int k = (int)tq;
    const v2u uk = ld2(ut, (uint32_t)k * 8u);
    const float a = fmaf(tq - (float)k, __uint_as_float(uk.y), __uint_as_float(uk.x)) - 0.5f;
    int i0 = (int)a;
    i0 = i0 > v.n_cols - 1 ? v.n_cols - 1 : (i0 < 0 ? 0 : i0);
    const int i1 = i0 + 1 < v.n_cols ? i0 + 1 : v.n_cols - 1;
    const float w = a - (float)i0;
    const float turns = angle_turns(dx, dy);
    const v2u c0 = ld2(ct, (uint32_t)i0 * 8u), c1 = ld2(ct, (uint32_t)i1 * 8u);
    int j00, j01, j10, j11;
    float t0, t1;
    column_rows((int)c0.x, turns, j00, j01, t0);
    column_rows((int)c1.x, turns, j10, j11, t1);
    const float4 A = ld4(lp, (c0.y + (uint32_t)j00) * 16u), B = ld4(lp, (c0.y + (uint32_t)j01) * 16u);
    const float4 C = ld4(lp, (c1.y + (uint32_t)j10) * 16u), D = ld4(lp, (c1.y + (uint32_t)j11) * 16u);
    const float w0 = 1.0f - w;
    return blend4(A, w0 - w0 * t0, B, w0 * t0, C, w - w * t1, D, w * t1);
}

__device__ __forceinline__ float4 sample_lmfr(const ReconView& v, float dx, float dy) {
    const __amdgpu_buffer_rsrc_t lp = rsrc(v.lp, v.lp_bytes);
    const float r = fmaxf(__builtin_amdgcn_sqrtf(fmaf(dx, dx, dy * dy)), 1.0f);
    const float z = __log2f(r) * v.inv_L;                     // Eq. (1); inv_L = ln 2 / L
    float u = (v.alpha == 4.0f ? (z * z) * (z * z) : __powf(z, v.alpha)) * (float)v.n_cols;   // Eq. (14)
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

// Pixel tile `id` of view v: 64 x R pixels, one per thread.  M is the
// mapping (kModeVafr / kModeLmfr) or -1 to read it from the view.
template <int R, int M>
__device__ __forceinline__ void recon_tile(const ReconView& v, int id) {
    const int nbx = (v.width + kTileW - 1) / kTileW, nby = (v.height + R - 1) / R;
    int bx, by;
    xcd_tile(id, nbx, nby, bx, by);
    const int x = bx * kTileW + (threadIdx.x & (kTileW - 1));
    const int ty = threadIdx.x / kTileW;
    const int y = by * R + ty;
    if (x >= v.width || y >= v.height) return;
    // offset of the pixel centre from the gaze point: film units for VaFR,
    // pixels for LMFR (cx, cy hold the gaze and the half-pixel shift)
    const float dx = fmaf((float)x, v.sx, v.cx), dy = fmaf((float)y, v.sy, v.cy);
    const int mode = M >= 0 ? M : v.mode;
    const float4 c = mode == kModeVafr ? sample_vafr(v, dx, dy) : sample_lmfr(v, dx, dy);
    // the tile's rows start at a uniform base; offsets stay 32-bit
    const __amdgpu_buffer_rsrc_t img = rsrc(v.img + (size_t)by * R * v.width, (uint32_t)(R * v.width) * 16u);
    store_px(img, (uint32_t)(ty * v.width + x) * 16u, c);
}

template <int R, int M>
__global__ __launch_bounds__(kTileW* R) void k_recon(const ReconView v) {
    recon_tile<R, M>(v, blockIdx.x);
}

// Batched launch over several views (block_end: running tile counts).
template <int R>
__global__ __launch_bounds__(kTileW* R) void k_recon_batch(const ReconView* __restrict__ views,
                                                         const int32_t* __restrict__ block_end, int32_t n_views) {
    const int b = blockIdx.x;
    int vid = 0;
    while (vid + 1 < n_views && b >= block_end[vid]) ++vid;
    const int first = vid ? block_end[vid - 1] : 0;
    recon_tile<R, -1>(views[vid], b - first);
}

}  // namespace

bool recon_rows_ok(int rows) { return rows == 1 || rows == 2 || rows == 4 || rows == 8; }

int64_t recon_blocks_of(const ReconView& v, int rows) {
    return (int64_t)((v.width + kTileW - 1) / kTileW) * ((v.height + rows - 1) / rows);
}

int launch_reconstruct(const ReconView& v, hipStream_t stream, int rows) {
    if (!recon_rows_ok(rows)) return fail(VAFR_E_ARG, "reconstruction tile height must be 1, 2, 4 or 8");
    const int64_t blocks = recon_blocks_of(v, rows);
    if (blocks > 0x7fffffff) return fail(VAFR_E_UNSUPPORTED, "display too large");
    const dim3 g((unsigned)blocks);
    if (v.mode == kModeVafr) {
        switch (rows) {
            case 1: hipLaunchKernelGGL((k_recon<1, kModeVafr>), g, dim3(kTileW * 1), 0, stream, v); break;
            case 2: hipLaunchKernelGGL((k_recon<2, kModeVafr>), g, dim3(kTileW * 2), 0, stream, v); break;
            case 4: hipLaunchKernelGGL((k_recon<4, kModeVafr>), g, dim3(kTileW * 4), 0, stream, v); break;
            default: hipLaunchKernelGGL((k_recon<8, kModeVafr>), g, dim3(kTileW * 8), 0, stream, v); break;
        }
    } else {
        switch (rows) {
            case 1: hipLaunchKernelGGL((k_recon<1, kModeLmfr>), g, dim3(kTileW * 1), 0, stream, v); break;
            case 2: hipLaunchKernelGGL((k_recon<2, kModeLmfr>), g, dim3(kTileW * 2), 0, stream, v); break;
            case 4: hipLaunchKernelGGL((k_recon<4, kModeLmfr>), g, dim3(kTileW * 4), 0, stream, v); break;
            default: hipLaunchKernelGGL((k_recon<8, kModeLmfr>), g, dim3(kTileW * 8), 0, stream, v); break;
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
    if (!recon_rows_ok(rows)) return fail(VAFR_E_ARG, "reconstruction tile height must be 1, 2, 4 or 8");
    const dim3 g((unsigned)blocks);
    switch (rows) {
        case 1: hipLaunchKernelGGL(k_recon_batch<1>, g, dim3(kTileW * 1), 0, stream, views_dev, block_end_dev, n_views); break;
        case 2: hipLaunchKernelGGL(k_recon_batch<2>, g, dim3(kTileW * 2), 0, stream, views_dev, block_end_dev, n_views); break;
        case 4: hipLaunchKernelGGL(k_recon_batch<4>, g, dim3(kTileW * 4), 0, stream, views_dev, block_end_dev, n_views); break;
        default: hipLaunchKernelGGL(k_recon_batch<8>, g, dim3(kTileW * 8), 0, stream, views_dev, block_end_dev, n_views); break;
    }
    VAFR_HIP(hipGetLastError());
    return VAFR_OK;
}

}  // namespace vafr
