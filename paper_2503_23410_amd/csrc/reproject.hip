// Binocular reprojection of the left LP buffer by forward grid warping
// (Sec. 5.1, VaFR_Rep: the right eye is warped from the left eye's LP buffer
// instead of being rendered a second time).
//
// The left texels' primary hit points form a grid mesh in LP topology: the
// band between columns s and s + 1 is triangulated by a zipper over the two
// columns' texels merged by angle (texel (i, j) sits at (2j + 1) / (2 n_i)
// turns; on equal angles the inner column first).  Texel x of column i
// closes two triangles, (previous texel of its column, x, last texel of the
// neighbouring column that precedes x in the merged order), id 2x + 1 in the
// band toward column i + 1 and 2x in the band toward column i - 1.
//
// Every vertex is projected into the right eye (FP32, fixed order); a
// triangle is dropped if a vertex did not hit, lies behind the eye or
// projects to a non-finite film point, its
// depths differ by more than 1/10, it is stretched to more than twice its
// left film size, or it has zero area: its area is then ray-cast.  A right
// texel whose sample point (gaze + film offset) lies inside a kept
// triangle (FP64 edge functions; an edge point belongs to both sides) gets
// the triangle's perspective-correct depth there, and the least (depth
// bits, triangle id) wins through a 64-bit atomic minimum.  A resolve pass
// writes the winners' interpolated colours and the hit id of the vertex of
// largest weight, and lists the uncovered texels in trace order so that the
// trace kernel ray-casts only those, with full waves.
//
// Candidate texels of a triangle come from its film bounding box mapped to
// LP coordinates (FP32, widened by bounds on the table and rounding errors
// so that no texel whose sample point lies in the box is missed); the exact
// FP64 test decides.  Built with -ffp-contract=off.
#include "vafr_internal.h"

namespace vafr {
namespace {

constexpr double kDepthRel = 0.1;   // largest depth ratio of a kept triangle, minus 1
constexpr double kStretch = 2.0;    // largest right / left film extent of a kept triangle

struct RightCam {
    float eye[3], right[3], up[3], fwd[3];
};

struct WarpView {
    int64_t n_texels;
    int32_t n_cols;
    const int2* col;          // (rows, first texel) per column
    const int32_t* blk_col;   // column of texel 256 b
    const float2* dxy;        // film offset per texel (texel order)
    const float2* u_of_rho;   // (u_k, u_{k+1} - u_k) at rho_k = k rho_max / kURhoN
    float rho_scale;          // kURhoN / rho_max
    float rho_max;
    float u_margin;           // bound on the table's error, in columns
    double gx, gy;            // gaze point on the film plane
    RightCam cam;
    const float4* points;     // left hit points (w = 1) or zeros
    unsigned long long* key;  // per right texel
};

struct ResolveView {
    WarpView w;
    const int32_t* ord;       // texel of each trace-order item
    RepBuffers b;
};

// Column of texel x: from the column of its 256-texel block, walk forward.
__device__ __forceinline__ int column_of_texel(const WarpView& v, int64_t x) {
    int c = v.blk_col[x / kTexelBlock];
    while (c + 1 < v.n_cols && (int64_t)v.col[c + 1].y <= x) ++c;
    return c;
}

// Last texel of the column with record co preceding texel (row j of a
// column of n rows) in the merged order; inner: whether co's column is the
// inner one of the band (it then wins ties).
__device__ __forceinline__ int64_t other_vertex(int2 co, int n, int j, bool inner) {
    const int64_t a = (int64_t)(2 * j + 1) * co.x;
    // inner column: (2k + 1) n <= a; outer column: (2k + 1) n < a
    const int64_t q = inner ? a / n : (a - 1) / n;
    const int64_t k = q == 0 ? (int64_t)co.x - 1 : (q - 1) / 2;
    return (int64_t)co.y + k;
}

// Vertex texels (previous, x, other) of triangle `side` of texel x = row j
// of column i; false when the band does not exist.
__device__ __forceinline__ bool triangle_vertices(const WarpView& v, int i, int j, int side, int64_t t[3]) {
    const int2 ci = v.col[i];
    const int o = side ? i + 1 : i - 1;
    if (o < 0 || o >= v.n_cols) return false;
    t[0] = (int64_t)ci.y + (j == 0 ? ci.x - 1 : j - 1);
    t[1] = (int64_t)ci.y + j;
    t[2] = other_vertex(v.col[o], ci.x, j, /*inner=*/side == 0);
    return true;
}

struct Vert {
    float fx, fy, z;
    bool ok;
};

// Right-eye film point and depth of a left hit point (FP32, fixed order).
__device__ __forceinline__ Vert project(const RightCam& c, float4 P) {
    Vert r{0.0f, 0.0f, 0.0f, false};
    if (P.w == 0.0f) return r;
    const float qx = P.x - c.eye[0], qy = P.y - c.eye[1], qz = P.z - c.eye[2];
    const float x = (qx * c.right[0] + qy * c.right[1]) + qz * c.right[2];
    const float y = (qx * c.up[0] + qy * c.up[1]) + qz * c.up[2];
    const float z = (qx * c.fwd[0] + qy * c.fwd[1]) + qz * c.fwd[2];
    if (!(z > 0.0f)) return r;
    r.fx = x / z;
    r.fy = -(y / z);
    r.z = z;
    r.ok = isfinite(r.fx) && isfinite(r.fy);
    return r;
}

__device__ __forceinline__ double edge(double px, double py, double qx, double qy, double cx, double cy) {
    return (qx - px) * (cy - py) - (qy - py) * (cx - px);
}

// Barycentric weights of sample point (cx, cy); false if outside.
__device__ __forceinline__ bool inside(const Vert* V, double A, double cx, double cy, double b[3]) {
    const double e0 = edge(V[1].fx, V[1].fy, V[2].fx, V[2].fy, cx, cy);
    const double e1 = edge(V[2].fx, V[2].fy, V[0].fx, V[0].fy, cx, cy);
    const double e2 = edge(V[0].fx, V[0].fy, V[1].fx, V[1].fy, cx, cy);
    const bool in = A > 0.0 ? (e0 >= 0.0 && e1 >= 0.0 && e2 >= 0.0) : (e0 <= 0.0 && e1 <= 0.0 && e2 <= 0.0);
    if (!in) return false;
    b[0] = e0 / A;
    b[1] = e1 / A;
    b[2] = e2 / A;
    return true;
}

__device__ __forceinline__ double inv_depth(const Vert* V, const double b[3]) {
    return (b[0] / (double)V[0].z + b[1] / (double)V[1].z) + b[2] / (double)V[2].z;
}

// Column coordinate (column centres at integers) of film radius rho.
__device__ __forceinline__ float column_coord(const WarpView& v, float rho) {
    const float tq = fminf(rho * v.rho_scale, (float)kURhoN);
    const int k = (int)tq;
    const float2 uk = v.u_of_rho[k];
    return fmaf(tq - (float)k, uk.y, uk.x) - 0.5f;
}

__global__ __launch_bounds__(256) void k_rep_clear(unsigned long long* key, int32_t* count, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < n) key[k] = ~0ull;
    if (k == 0) *count = 0;
}

// One thread per left texel: its two triangles.
__global__ __launch_bounds__(kTexelBlock) void k_rep_warp(const WarpView v) {
    const int64_t x = (int64_t)blockIdx.x * kTexelBlock + threadIdx.x;
    if (x >= v.n_texels) return;
    const int i = column_of_texel(v, x);
    const int j = (int)(x - v.col[i].y);
    for (int side = 0; side < 2; ++side) {
        int64_t t[3];
        if (!triangle_vertices(v, i, j, side, t)) continue;
        Vert V[3];
        bool ok = true;
        for (int c = 0; c < 3; ++c) {
            V[c] = project(v.cam, v.points[t[c]]);
            ok = ok && V[c].ok;
        }
        if (!ok) continue;
        const float zmin = fminf(fminf(V[0].z, V[1].z), V[2].z), zmax = fmaxf(fmaxf(V[0].z, V[1].z), V[2].z);
        if ((double)zmax > (double)zmin * (1.0 + kDepthRel)) continue;
        double rx0 = V[0].fx, rx1 = V[0].fx, ry0 = V[0].fy, ry1 = V[0].fy;
        double lx0 = INFINITY, lx1 = -INFINITY, ly0 = INFINITY, ly1 = -INFINITY;
        for (int c = 0; c < 3; ++c) {
            rx0 = fmin(rx0, (double)V[c].fx);
            rx1 = fmax(rx1, (double)V[c].fx);
            ry0 = fmin(ry0, (double)V[c].fy);
            ry1 = fmax(ry1, (double)V[c].fy);
            const float2 o = v.dxy[t[c]];
            const double X = v.gx + (double)o.x, Y = v.gy + (double)o.y;
            lx0 = fmin(lx0, X);
            lx1 = fmax(lx1, X);
            ly0 = fmin(ly0, Y);
            ly1 = fmax(ly1, Y);
        }
        if (fmax(rx1 - rx0, ry1 - ry0) > kStretch * fmax(lx1 - lx0, ly1 - ly0)) continue;
        const double A = edge(V[0].fx, V[0].fy, V[1].fx, V[1].fy, V[2].fx, V[2].fy);
        if (A == 0.0) continue;
        const unsigned long long id = (unsigned long long)(2 * x + side);
        // candidate texels: the box relative to the gaze in LP coordinates
        const float ox0 = (float)(rx0 - v.gx), ox1 = (float)(rx1 - v.gx);
        const float oy0 = (float)(ry0 - v.gy), oy1 = (float)(ry1 - v.gy);
        const float cx = ox0 > 0.0f ? ox0 : (ox1 < 0.0f ? -ox1 : 0.0f);
        const float cy = oy0 > 0.0f ? oy0 : (oy1 < 0.0f ? -oy1 : 0.0f);
        const float rho_lo = sqrtf(cx * cx + cy * cy);
        if (rho_lo > v.rho_max * 1.001f) continue;
        const float mx = fmaxf(ox0 * ox0, ox1 * ox1), my = fmaxf(oy0 * oy0, oy1 * oy1);
        const float rho_hi = sqrtf(mx + my);
        const int i0 = max(0, (int)ceilf(column_coord(v, rho_lo) - v.u_margin));
        const int i1 = min(v.n_cols - 1, (int)floorf(column_coord(v, rho_hi) + v.u_margin));
        const bool all_angles = ox0 <= 0.0f && ox1 >= 0.0f && oy0 <= 0.0f && oy1 >= 0.0f;
        // angular margin (turns): film coordinates within 4e-7 of the exact
        // ones seen from radius rho_lo, plus atan2f's error
        const float slop = (4e-7f / fmaxf(rho_lo, 1e-30f) + 4e-6f) * (0.5f / (float)M_PI);
        float t0 = 0.0f, t1 = 1.0f;
        if (!all_angles) {
            const float pc = atan2f(0.5f * (oy0 + oy1), 0.5f * (ox0 + ox1));
            float dlo = 0.0f, dhi = 0.0f;
            const float qx[4] = {ox0, ox1, ox0, ox1}, qy[4] = {oy0, oy0, oy1, oy1};
            for (int q = 0; q < 4; ++q) {
                float d = atan2f(qy[q], qx[q]) - pc;
                if (d > (float)M_PI) d -= 2.0f * (float)M_PI;
                if (d < -(float)M_PI) d += 2.0f * (float)M_PI;
                dlo = fminf(dlo, d);
                dhi = fmaxf(dhi, d);
            }
            t0 = (pc + dlo) * (0.5f / (float)M_PI);
            t1 = (pc + dhi) * (0.5f / (float)M_PI);
        }
        for (int ci = i0; ci <= i1; ++ci) {
            const int2 cc = v.col[ci];
            const int n = cc.x;
            int j0 = 0, cnt = n;
            if (!all_angles) {
                const float m = fminf(slop * (float)n + 0.01f, (float)n);
                j0 = (int)ceilf(t0 * (float)n - 0.5f - m);
                cnt = (int)floorf(t1 * (float)n - 0.5f + m) - j0 + 1;
                if (!(cnt < n)) {
                    j0 = 0;
                    cnt = n;
                }
            }
            int jj = j0 % n;
            if (jj < 0) jj += n;
            for (int r = 0; r < cnt; ++r) {
                const int64_t c = (int64_t)cc.y + jj;
                if (++jj == n) jj = 0;
                const float2 o = v.dxy[c];
                const double px = v.gx + (double)o.x, py = v.gy + (double)o.y;
                double b[3];
                if (!inside(V, A, px, py, b)) continue;
                const float depth = (float)(1.0 / inv_depth(V, b));
                atomicMin(v.key + c, ((unsigned long long)__float_as_uint(depth) << 32) | id);
            }
        }
    }
}

// One thread per trace-order item: a covered texel takes its triangle's
// interpolated colour; the workgroup's uncovered items are appended to the
// hole list as one contiguous run, in item order (one atomic per workgroup).
__global__ __launch_bounds__(256) void k_rep_resolve(const ResolveView r) {
    __shared__ int wave_n[4];
    __shared__ int run_base;
    const WarpView& v = r.w;
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool hole = false;
    if (k < v.n_texels) {
        const int32_t t = r.ord[k];
        const unsigned long long key = v.key[t];
        if (key == ~0ull) {
            hole = true;
        } else {
            const int64_t tri = (int64_t)(uint32_t)key;
            const int64_t x = tri >> 1;
            const int i = column_of_texel(v, x);
            int64_t tv[3];
            triangle_vertices(v, i, (int)(x - v.col[i].y), (int)(tri & 1), tv);
            Vert V[3];
            for (int c = 0; c < 3; ++c) V[c] = project(v.cam, v.points[tv[c]]);
            const double A = edge(V[0].fx, V[0].fy, V[1].fx, V[1].fy, V[2].fx, V[2].fy);
            const float2 o = v.dxy[t];
            double b[3] = {1.0, 0.0, 0.0};
            inside(V, A, v.gx + (double)o.x, v.gy + (double)o.y, b);
            const double s = inv_depth(V, b);
            double w[3];
            for (int c = 0; c < 3; ++c) w[c] = (b[c] / (double)V[c].z) / s;
            const float4 c0 = r.b.src_rgba[tv[0]], c1 = r.b.src_rgba[tv[1]], c2 = r.b.src_rgba[tv[2]];
            r.b.out_rgba[t] = make_float4(
                (float)((w[0] * (double)c0.x + w[1] * (double)c1.x) + w[2] * (double)c2.x),
                (float)((w[0] * (double)c0.y + w[1] * (double)c1.y) + w[2] * (double)c2.y),
                (float)((w[0] * (double)c0.z + w[1] * (double)c1.z) + w[2] * (double)c2.z),
                (float)((w[0] * (double)c0.w + w[1] * (double)c1.w) + w[2] * (double)c2.w));
            if (r.b.out_id) {
                int top = 0;
                if (w[1] > w[top]) top = 1;
                if (w[2] > w[top]) top = 2;
                r.b.out_id[t] = r.b.src_id ? r.b.src_id[tv[top]] : -1;
            }
        }
    }
    const unsigned long long m = __ballot(hole);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int below = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wave_n[wv] = __popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        const int n = (wave_n[0] + wave_n[1]) + (wave_n[2] + wave_n[3]);
        run_base = n ? atomicAdd(r.b.count, n) : 0;
    }
    __syncthreads();
    if (hole) {
        int off = run_base + below;
        for (int q = 0; q < wv; ++q) off += wave_n[q];
        r.b.list[off] = (int32_t)k;
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
    WarpView v;
    v.n_texels = n;
    v.n_cols = L.n_cols;
    v.col = ld.col;
    v.blk_col = ld.blk_col;
    v.dxy = ld.dxy_tex;
    v.u_of_rho = ld.u_of_rho;
    v.rho_scale = (float)(kURhoN / L.rho_max);
    v.rho_max = (float)L.rho_max;
    v.u_margin = (float)L.u_margin;
    v.gx = gx;
    v.gy = gy;
    for (int c = 0; c < 3; ++c) {
        v.cam.eye[c] = right.eye[c];
        v.cam.right[c] = right.right[c];
        v.cam.up[c] = right.up[c];
        v.cam.fwd[c] = right.forward[c];
    }
    v.points = b.points;
    v.key = b.key;
    static_assert(kTexelBlock == 256, "texel kernels use 256-texel workgroups");
    hipLaunchKernelGGL(k_rep_warp, dim3(blocks), dim3(kTexelBlock), 0, stream, v);
    VAFR_HIP(hipGetLastError());
    ResolveView r{v, ld.ord, b};
    hipLaunchKernelGGL(k_rep_resolve, dim3(blocks), dim3(256), 0, stream, r);
    VAFR_HIP(hipGetLastError());
    return VAFR_OK;
}

}  // namespace vafr
