// Binocular reprojection from the left LP buffer (Sec. 5.1, VaFR_Rep: the
// right eye reuses the left eye's LP buffer instead of being rendered a
// second time).
//
// Every left texel whose primary ray hit carries its hit point into the right
// eye: the point is projected onto the right film plane (FP32, operation
// order fixed below), mapped to the LP cell that holds it (FP64: Eq. (3)
// radius -> eccentricity, Eq. (5) / Eq. (12) abscissa, and the polar angle;
// row j of column i covers angles 360 j / n_i .. 360 (j + 1) / n_i), and
// competes for that cell with a 64-bit atomic minimum of (depth bits << 32 |
// left texel): the nearest point wins, then the lower left texel.  A resolve
// pass then copies each winner's colour and hit id into the right buffers
// and lists the cells nobody reached, in trace order, so that the trace
// kernel ray-casts only those, with full waves.  Built with
// -ffp-contract=off.
#include "vafr_internal.h"

namespace vafr {
namespace {

struct RepView {
    int64_t n_texels;
    int32_t n_cols;
    const int2* col;          // (rows, first texel) per column
    Segments seg;             // FP64 acuity segments of the layout
    double gx, gy;            // gaze point on the film plane
    float eye[3], right[3], up[3], fwd[3];   // right-eye camera
    const float4* points;     // left hit points (w = 1) or zeros
    unsigned long long* key;  // per right texel
};

struct ResolveView {
    int64_t n_texels;
    const int32_t* ord;       // texel of each trace-order item
    RepBuffers b;
};

// Eq. (5) on the segment holding e (the last segment extends beyond it).
__device__ __forceinline__ double abscissa(const Segments& s, double e) {
    int k = 0;
    while (k + 1 < s.n && e >= s.e[k + 1]) ++k;
    if (s.m[k] == 0.0) return 2.0 * e / s.b[k] + s.c[k];
    return 2.0 * log(s.m[k] * e + s.b[k]) / s.m[k] + s.c[k];
}

__global__ __launch_bounds__(256) void k_rep_clear(unsigned long long* key, int32_t* count, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < n) key[k] = ~0ull;
    if (k == 0) *count = 0;
}

__global__ __launch_bounds__(256) void k_rep_splat(const RepView v) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= v.n_texels) return;
    const float4 P = v.points[k];
    if (P.w == 0.0f) return;
    const float qx = P.x - v.eye[0], qy = P.y - v.eye[1], qz = P.z - v.eye[2];
    const float x = (qx * v.right[0] + qy * v.right[1]) + qz * v.right[2];
    const float y = (qx * v.up[0] + qy * v.up[1]) + qz * v.up[2];
    const float z = (qx * v.fwd[0] + qy * v.fwd[1]) + qz * v.fwd[2];
    if (!(z > 0.0f)) return;
    const float fx = x / z, fy = -(y / z);
    const double dx = (double)fx - v.gx, dy = (double)fy - v.gy;
    const double rho = sqrt(dx * dx + dy * dy);
    const double e = atan(rho) / (M_PI / 180.0);
    const double u = abscissa(v.seg, e);
    if (!(u < (double)v.n_cols)) return;                 // beyond the last column
    const int i = (int)floor(u);
    double th = atan2(dy, dx) / (M_PI / 180.0);
    if (th < 0.0) th += 360.0;
    const int2 c = v.col[i];
    int j = (int)floor(th / 360.0 * (double)c.x);
    if (j >= c.x) j = c.x - 1;
    const unsigned long long kk = ((unsigned long long)__float_as_uint(z) << 32) | (unsigned long long)(uint32_t)k;
    atomicMin(v.key + c.y + j, kk);
}

// One thread per trace-order item: a reached cell takes its winner; the
// workgroup's unreached items are appended to the hole list as one
// contiguous run, in item order (one atomic per workgroup).
__global__ __launch_bounds__(256) void k_rep_resolve(const ResolveView v) {
    __shared__ int wave_n[4];
    __shared__ int run_base;
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool hole = false;
    if (k < v.n_texels) {
        const int32_t t = v.ord[k];
        const unsigned long long key = v.b.key[t];
        if (key == ~0ull) {
            hole = true;
        } else {
            const uint32_t src = (uint32_t)key;
            v.b.out_rgba[t] = v.b.src_rgba[src];
            if (v.b.out_id) v.b.out_id[t] = v.b.src_id ? v.b.src_id[src] : -1;
        }
    }
    const unsigned long long m = __ballot(hole);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int below = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wave_n[w] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int n = (wave_n[0] + wave_n[1]) + (wave_n[2] + wave_n[3]);
        run_base = n ? atomicAdd(v.b.count, n) : 0;
    }
    __syncthreads();
    if (hole) {
        int off = run_base + below;
        for (int q = 0; q < w; ++q) off += wave_n[q];
        v.b.list[off] = (int32_t)k;
    }
}

}  // namespace

int launch_rep(const LayoutDev& ld, const vafr_layout_s& L, double gx, double gy, const vafr_camera& right,
               const RepBuffers& b, hipStream_t stream) {
    const int64_t n = L.n_texels;
    if (n <= 0) return VAFR_OK;
    if (n > 0x7fffffff) return fail(VAFR_E_UNSUPPORTED, "too many texels for reprojection");
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_rep_clear, dim3(blocks), dim3(256), 0, stream, b.key, b.count, n);
    VAFR_HIP(hipGetLastError());
    RepView v;
    v.n_texels = n;
    v.n_cols = L.n_cols;
    v.col = ld.col;
    v.seg = L.seg;
    v.gx = gx;
    v.gy = gy;
    for (int c = 0; c < 3; ++c) {
        v.eye[c] = right.eye[c];
        v.right[c] = right.right[c];
        v.up[c] = right.up[c];
        v.fwd[c] = right.forward[c];
    }
    v.points = b.points;
    v.key = b.key;
    hipLaunchKernelGGL(k_rep_splat, dim3(blocks), dim3(256), 0, stream, v);
    VAFR_HIP(hipGetLastError());
    ResolveView r{n, ld.ord, b};
    hipLaunchKernelGGL(k_rep_resolve, dim3(blocks), dim3(256), 0, stream, r);
    VAFR_HIP(hipGetLastError());
    return VAFR_OK;
}

}  // namespace vafr
