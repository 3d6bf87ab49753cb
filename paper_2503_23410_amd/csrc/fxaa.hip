// FXAA-style edge anti-aliasing inside the VaFR LP buffer (Sec. 3.4: the
// LP buffer is anti-aliased before the inverse map, because in the
// periphery one texel covers many display pixels).
//
// The method of Lottes (FXAA, 2009) is applied on the ragged polar grid:
// along the angle a texel's neighbours are the adjacent rows of its column
// (cyclic); along the radius they are the inner and outer columns sampled at
// the texel's angle, linear in the row coordinate.  Per texel: a luma
// contrast test, the edge normal from second differences, the side of the
// edge with the larger luma step, a search for the two ends of the edge
// along it, a sub-texel term, and a blend toward the neighbour across the
// edge.  The constants and the operation order (FP32, no fused multiply-add;
// built with -ffp-contract=off) are part of the library's contract with its
// test oracle.
//
// One thread per texel.  The kernel reads the LP buffer through the caches
// (17 MB per view): a texel and its direct neighbours come from the same or
// adjacent columns, contiguous in the buffer for consecutive rows.
#include "vafr_internal.h"

namespace vafr {
namespace {

constexpr float kEdgeRel = 0.125f;   // contrast threshold relative to the local luma maximum
constexpr float kEdgeMin = 0.0625f;  // absolute contrast threshold
constexpr float kSubpix = 0.75f;     // weight of the sub-texel term
constexpr int kSteps = 6;
__constant__ float kStepAt[kSteps] = {1.0f, 2.0f, 3.0f, 4.0f, 6.0f, 8.0f};   // end-search offsets

struct FxaaView {
    const int2* col;     // (rows, first texel) per column
    const int32_t* blk_col;   // column of the first texel of each workgroup
    int32_t n_cols;
    int64_t n_texels;
    const float4* in;
    float4* out;
};

// Row j (any integer, cyclic) of the column with record cn = (rows, first
// texel); the modulo is only taken when j leaves [0, rows).
__device__ __forceinline__ float4 texel_of(const FxaaView& v, int2 cn, int j) {
    int r = j;
    if ((unsigned)r >= (unsigned)cn.x) {
        r = j % cn.x;
        r = r < 0 ? r + cn.x : r;
    }
    return v.in[(int64_t)cn.y + r];
}

__device__ __forceinline__ int clamp_col(const FxaaView& v, int c) {
    return c < 0 ? 0 : (c >= v.n_cols ? v.n_cols - 1 : c);
}

// The column with record cn at angle t turns, linear between rows.
__device__ __forceinline__ float4 column_of(const FxaaView& v, int2 cn, float t) {
    const float s = t * (float)cn.x - 0.5f;
    const float fs = floorf(s);
    const float w = s - fs;
    const int j0 = (int)fs;
    const float4 a = texel_of(v, cn, j0), b = texel_of(v, cn, j0 + 1);
    return make_float4(a.x + w * (b.x - a.x), a.y + w * (b.y - a.y), a.z + w * (b.z - a.z), a.w + w * (b.w - a.w));
}

// Column c (clamped to the buffer) at angle t turns.
__device__ __forceinline__ float4 column_at(const FxaaView& v, int c, float t) {
    return column_of(v, v.col[clamp_col(v, c)], t);
}

__device__ __forceinline__ float luma(float4 p) { return (0.299f * p.x + 0.587f * p.y) + 0.114f * p.z; }

// |second difference| of three lumas along a line.
__device__ __forceinline__ float curvature(float a, float m, float b) { return fabsf((a - m) + (b - m)); }

__device__ float4 fxaa_texel(const FxaaView& v, int i, int j) {
    // records of the texel's column and of its outer and inner neighbours
    const int2 ci = v.col[i], co = v.col[clamp_col(v, i + 1)], cn = v.col[clamp_col(v, i - 1)];
    const int n = ci.x;
    const float t = ((float)j + 0.5f) / (float)n;
    const float dt = 1.0f / (float)n;
    const float4 M = texel_of(v, ci, j);
    const float lM = luma(M);
    const float lU = luma(texel_of(v, ci, j + 1)), lD = luma(texel_of(v, ci, j - 1));
    const float lO = luma(column_of(v, co, t)), lI = luma(column_of(v, cn, t));
    const float lmax = fmaxf(fmaxf(fmaxf(lM, lU), fmaxf(lD, lO)), lI);
    const float lmin = fminf(fminf(fminf(lM, lU), fminf(lD, lO)), lI);
    const float range = lmax - lmin;
    if (range < fmaxf(kEdgeMin, lmax * kEdgeRel)) return M;
    const float lOU = luma(column_of(v, co, t + dt)), lOD = luma(column_of(v, co, t - dt));
    const float lIU = luma(column_of(v, cn, t + dt)), lID = luma(column_of(v, cn, t - dt));
    // luma curvature across the radius (three angles) and across the angle
    // (three radii), centre line weighted twice
    const float across_r = (curvature(lID, lD, lOD) + 2.0f * curvature(lI, lM, lO)) + curvature(lIU, lU, lOU);
    const float across_a = (curvature(lID, lI, lIU) + 2.0f * curvature(lD, lM, lU)) + curvature(lOD, lO, lOU);
    const bool radial = across_r >= across_a;   // the normal of the edge points along the radius
    const float lNeg = radial ? lI : lD, lPos = radial ? lO : lU;
    const float gNeg = fabsf(lNeg - lM), gPos = fabsf(lPos - lM);
    const int side = gPos >= gNeg ? 1 : -1;
    const float lSide = side > 0 ? lPos : lNeg;
    const float lLine = 0.5f * (lM + lSide);
    const float gScaled = 0.25f * fmaxf(gNeg, gPos);
    float dist[2], lEnd[2];
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
        const float sgn = dir == 0 ? -1.0f : 1.0f;
        dist[dir] = kStepAt[kSteps - 1] + 1.0f;
        lEnd[dir] = lLine;
        for (int k = 0; k < kSteps; ++k) {
            const float p = sgn * kStepAt[k];
            float la, lb;
            if (radial) {
                const float tt = t + p * dt;
                la = luma(column_of(v, ci, tt));
                lb = luma(column_of(v, side > 0 ? co : cn, tt));
            } else {
                const int c = i + (int)p;
                la = luma(column_at(v, c, t));
                lb = luma(column_at(v, c, t + (float)side * dt));
            }
            const float l = 0.5f * (la + lb);
            if (fabsf(l - lLine) >= gScaled) {
                dist[dir] = kStepAt[k];
                lEnd[dir] = l;
                break;
            }
        }
    }
    const int near = dist[0] <= dist[1] ? 0 : 1;
    const bool centre_below = lM - lLine < 0.0f, end_below = lEnd[near] - lLine < 0.0f;
    const float edge = centre_below != end_below ? 0.5f - dist[near] / (dist[0] + dist[1]) : 0.0f;
    const float lAvg = (2.0f * ((lU + lD) + (lI + lO)) + ((lIU + lID) + (lOU + lOD))) / 12.0f;
    const float s1 = fminf(fmaxf(fabsf(lAvg - lM) / range, 0.0f), 1.0f);
    const float s2 = (-2.0f * s1 + 3.0f) * (s1 * s1);
    const float off = fmaxf(edge, (s2 * s2) * kSubpix);
    const float4 S = radial ? column_of(v, side > 0 ? co : cn, t) : texel_of(v, ci, j + side);
    return make_float4(M.x + off * (S.x - M.x), M.y + off * (S.y - M.y), M.z + off * (S.z - M.z),
                       M.w + off * (S.w - M.w));
}

__global__ __launch_bounds__(kTexelBlock) void k_fxaa(const FxaaView v) {
    const int64_t k = (int64_t)blockIdx.x * kTexelBlock + threadIdx.x;
    if (k >= v.n_texels) return;
    // column of texel k: from the workgroup's first column, walk forward
    // (a workgroup spans several columns only near the centre of the grid)
    int c = v.blk_col[blockIdx.x];
    while (c + 1 < v.n_cols && (int64_t)v.col[c + 1].y <= k) ++c;
    v.out[k] = fxaa_texel(v, c, (int)(k - v.col[c].y));
}

}  // namespace

int launch_fxaa(const int2* col_dev, const int32_t* blk_col_dev, int32_t n_cols, int64_t n_texels, const float* in,
                float* out, hipStream_t stream) {
    if (n_texels <= 0) return VAFR_OK;
    FxaaView v{col_dev, blk_col_dev, n_cols, n_texels, reinterpret_cast<const float4*>(in),
               reinterpret_cast<float4*>(out)};
    const int64_t blocks = (n_texels + kTexelBlock - 1) / kTexelBlock;
    hipLaunchKernelGGL(k_fxaa, dim3((unsigned)blocks), dim3(kTexelBlock), 0, stream, v);
    VAFR_HIP(hipGetLastError());
    return VAFR_OK;
}

}  // namespace vafr
