// Inverse mapping of the LP buffer onto the display (Sec. 3.2.3,
// Eqs. (10)-(11)), one thread per display pixel.
//
// Each wave covers 64 consecutive pixels of one display row, so the 16-byte
// RGBA stores of a wave form one contiguous 1 KiB segment; they are
// non-temporal because the image is written once and not read back here.
// The LP buffer (17 MB per VaFR view) is read through the caches: a texel
// feeds tens of display pixels in the periphery.
//
// Workgroups are mapped XCD-aware: consecutive workgroup ids land on
// different XCDs, so the id is permuted such that each XCD receives a
// contiguous band of display rows and reads a compact part of the LP buffer
// through its own L2.
#include "vafr_internal.h"

namespace vafr {
namespace {

constexpr int kTileW = 64;
constexpr int kTileH = 4;
constexpr int kXcds = 8;

// Workgroup id -> (tile x, tile y) so that XCD q (= id mod 8) gets the q-th
// contiguous eighth of the tiles in row-major order.
__device__ __forceinline__ void xcd_tile(int nbx, int nby, int& bx, int& by) {
    const int n = nbx * nby;
    const int id = blockIdx.x;
    int t = id;
    if (n >= kXcds * 64) {
        const int per = n / kXcds;              // tiles per XCD (full part)
        const int full = per * kXcds;
        if (id < full) t = (id % kXcds) * per + id / kXcds;
    }
    bx = t % nbx;
    by = t / nbx;
}

typedef float v4f __attribute__((ext_vector_type(4)));

// Streaming 16-byte store of one pixel.
__device__ __forceinline__ void store_px(float4* dst, float4 c) {
    v4f v = {c.x, c.y, c.z, c.w};
    __builtin_nontemporal_store(v, reinterpret_cast<v4f*>(dst));
}

__device__ __forceinline__ float4 lerp4(float4 a, float4 b, float t) {
    const float s = 1.0f - t;
    return make_float4(s * a.x + t * b.x, s * a.y + t * b.y, s * a.z + t * b.z, s * a.w + t * b.w);
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
    float r = p * a;                                          // [0, pi/4]
    r = ay > ax ? 1.5707963267948966f - r : r;
    r = dx < 0.0f ? 3.141592653589793f - r : r;
    r = dy < 0.0f ? 6.283185307179586f - r : r;
    return r * 0.15915494309189535f;
}

// Angular interpolation inside one column (n rows starting at off), at
// angle `turns` (fraction of the full circle).
__device__ __forceinline__ float4 column_sample(const float4* __restrict__ lp, int2 col, float turns) {
    const int n = col.x;
    const float s = fmaf(turns, (float)n, -0.5f);
    const float fs = floorf(s);
    const float t = s - fs;
    int j0 = (int)fs;
    j0 = j0 < 0 ? j0 + n : (j0 >= n ? j0 - n : j0);
    const int j1 = j0 + 1 == n ? 0 : j0 + 1;
    return lerp4(lp[col.y + j0], lp[col.y + j1], t);
}

__global__ __launch_bounds__(kTileW* kTileH) void k_recon_vafr(const ReconVafr R) {
    const int nbx = (R.width + kTileW - 1) / kTileW, nby = (R.height + kTileH - 1) / kTileH;
    int bx, by;
    xcd_tile(nbx, nby, bx, by);
    const int x = bx * kTileW + (threadIdx.x & (kTileW - 1));
    const int y = by * kTileH + (threadIdx.x / kTileW);
    if (x >= R.width || y >= R.height) return;
    const float X = ((float)x + 0.5f - 0.5f * (float)R.width) * R.px;
    const float Y = ((float)y + 0.5f - 0.5f * (float)R.height) * R.py;
    const float dx = X - R.gx, dy = Y - R.gy;
    const float rho = __builtin_amdgcn_sqrtf(fmaf(dx, dx, dy * dy));
    // u(e(rho)) (Eqs. (3), (5), (12)) from the FP64-built radial table,
    // already clamped to the first and last column centres.
    const float tq = fminf(rho * R.rho_scale, (float)kURhoN);
    const int k = (int)tq;
    const float2 uk = R.u_of_rho[k];
    const float u = fmaf(tq - (float)k, uk.y, uk.x);
    const float a = u - 0.5f;
    int i0 = (int)a;
    i0 = i0 > R.n_cols - 1 ? R.n_cols - 1 : (i0 < 0 ? 0 : i0);
    const int i1 = i0 + 1 < R.n_cols ? i0 + 1 : R.n_cols - 1;
    const float w = a - (float)i0;
    const float turns = angle_turns(dx, dy);
    const float4 c0 = column_sample(R.lp, R.col[i0], turns);
    const float4 c1 = column_sample(R.lp, R.col[i1], turns);
    store_px(R.img + (size_t)y * R.width + x, lerp4(c0, c1, w));
}

__global__ __launch_bounds__(kTileW* kTileH) void k_recon_lmfr(const ReconLmfr R) {
    const int nbx = (R.width + kTileW - 1) / kTileW, nby = (R.height + kTileH - 1) / kTileH;
    int bx, by;
    xcd_tile(nbx, nby, bx, by);
    const int x = bx * kTileW + (threadIdx.x & (kTileW - 1));
    const int y = by * kTileH + (threadIdx.x / kTileW);
    if (x >= R.width || y >= R.height) return;
    const float dx = (float)x + 0.5f - R.gx, dy = (float)y + 0.5f - R.gy;
    const float r = fmaxf(sqrtf(dx * dx + dy * dy), 1.0f);
    const float z = __log2f(r) * R.inv_L;                     // Eq. (1); inv_L = ln 2 / L
    float u = (R.alpha == 4.0f ? (z * z) * (z * z) : __powf(z, R.alpha)) * (float)R.w;   // Eq. (14)
    const float v = angle_turns(dx, dy) * (float)R.h;
    u = fminf(fmaxf(u, 0.5f), (float)R.w - 0.5f);
    const float a = u - 0.5f;
    int i0 = (int)a;
    i0 = i0 > R.w - 1 ? R.w - 1 : i0;
    const int i1 = i0 + 1 < R.w ? i0 + 1 : R.w - 1;
    const float wc = a - (float)i0;
    const float s = v - 0.5f;
    const float fs = floorf(s);
    const float t = s - fs;
    int j0 = (int)fs;
    j0 = j0 < 0 ? j0 + R.h : (j0 >= R.h ? j0 - R.h : j0);
    const int j1 = j0 + 1 == R.h ? 0 : j0 + 1;
    const size_t o0 = (size_t)i0 * R.h, o1 = (size_t)i1 * R.h;
    const float4 c0 = lerp4(R.lp[o0 + j0], R.lp[o0 + j1], t);
    const float4 c1 = lerp4(R.lp[o1 + j0], R.lp[o1 + j1], t);
    store_px(R.img + (size_t)y * R.width + x, lerp4(c0, c1, wc));
}

dim3 recon_grid(int W, int H) {
    const int nbx = (W + kTileW - 1) / kTileW, nby = (H + kTileH - 1) / kTileH;
    return dim3((unsigned)(nbx * nby));
}

}  // namespace

int launch_reconstruct_vafr(const ReconVafr& r, hipStream_t stream) {
    hipLaunchKernelGGL(k_recon_vafr, recon_grid(r.width, r.height), dim3(kTileW * kTileH), 0, stream, r);
    VAFR_HIP(hipGetLastError());
    return VAFR_OK;
}

int launch_reconstruct_lmfr(const ReconLmfr& r, hipStream_t stream) {
    hipLaunchKernelGGL(k_recon_lmfr, recon_grid(r.width, r.height), dim3(kTileW * kTileH), 0, stream, r);
    VAFR_HIP(hipGetLastError());
    return VAFR_OK;
}

}  // namespace vafr
