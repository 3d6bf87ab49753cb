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
constexpr float kRadToDeg = 57.29577951308232f;

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

__device__ __forceinline__ float theta_deg(float dx, float dy) {
    float th = atan2f(dy, dx) * kRadToDeg;
    return th < 0.0f ? th + 360.0f : th;
}

// Angular interpolation inside one column of n rows starting at off.
__device__ __forceinline__ float4 column_sample(const float4* __restrict__ lp, int2 col, float th) {
    const int n = col.x;
    const float s = th * ((float)n * (1.0f / 360.0f)) - 0.5f;
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
    const float rho = sqrtf(dx * dx + dy * dy);
    const float e = atanf(rho) * kRadToDeg;                 // Eq. (3)
    const float th = theta_deg(dx, dy);
    // Eq. (5) on the segment holding e (Eq. (12)); segment constants are
    // uniform, so the scan reads them with scalar loads.
    float m = R.seg.m[0], b = R.seg.b[0], tm = R.seg.two_over_m[0], c = R.seg.c[0];
    for (int q = 1; q < R.seg.n; ++q) {
        if (e >= R.seg.e[q]) { m = R.seg.m[q]; b = R.seg.b[q]; tm = R.seg.two_over_m[q]; c = R.seg.c[q]; }
    }
    float u = m != 0.0f ? tm * __logf(fmaf(m, e, b)) + c : 2.0f * e / b + c;
    u = fminf(fmaxf(u, 0.5f), (float)R.n_cols - 0.5f);
    const float a = u - 0.5f;
    int i0 = (int)a;
    i0 = i0 > R.n_cols - 1 ? R.n_cols - 1 : i0;
    const int i1 = i0 + 1 < R.n_cols ? i0 + 1 : R.n_cols - 1;
    const float w = a - (float)i0;
    const float4 c0 = column_sample(R.lp, R.col[i0], th);
    const float4 c1 = column_sample(R.lp, R.col[i1], th);
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
    const float z = __logf(r) * R.inv_L;                      // Eq. (1)
    float u = (R.alpha == 4.0f ? (z * z) * (z * z) : __powf(z, R.alpha)) * (float)R.w;   // Eq. (14)
    const float v = theta_deg(dx, dy) * ((float)R.h * (1.0f / 360.0f));
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
