// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <deque>
#include <mutex>
#include <string>
#include <vector>

#include "vafr.h"

namespace vafr {

// ------------------------------------------------------------------ errors
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
#define VAFR_HIP(call)                                      \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return ::vafr::hip_fail(e_, #call); \
    } while (0)

// ------------------------------------------------------- acuity segments
// MAR omega(e) = m_k e + b_k on [e_k, e_{k+1}); u(e) = 2 ln(omega)/m_k + c_k.
constexpr int kMaxSeg = 16;
struct Segments {
    int n = 0;
    double e[kMaxSeg + 1] = {};
    double m[kMaxSeg] = {};
    double b[kMaxSeg] = {};
    double c[kMaxSeg] = {};
    double u[kMaxSeg + 1] = {};
};

// Size of the radial table u(rho) used by the reconstruction kernel.
constexpr int kURhoN = 16384;

// Per-device copy of a layout's tables.
struct LayoutDev {
    int device = -1;
    int2* col = nullptr;          // VaFR: (n_rows, col_off) per column
    float2* dxy = nullptr;        // VaFR: film offset per texel, in trace order
    float2* dxy_tex = nullptr;    // VaFR: film offset per texel, in texel order
    int32_t* ord = nullptr;       // VaFR: texel index of each trace-order slot
    int32_t* blk_col = nullptr;   // VaFR: column of texel 256 b (per-texel kernels' block start)
    float2* u_of_rho = nullptr;   // VaFR: (u_k, u_{k+1} - u_k) at rho_k = k h, k <= kURhoN
    double* lm_z = nullptr;       // LMFR: z_i per column
    double2* lm_cs = nullptr;     // LMFR: (cos, sin) of theta_j per row
};

}  // namespace vafr

struct vafr_layout_s {
    int kind = VAFR_LAYOUT_VAFR;
    vafr_display disp{};
    double px = 0, py = 0;               // film pitch per pixel (FP64)
    // VaFR
    vafr::Segments seg;
    double e_max = 60.0;
    std::vector<double> aniso_e, aniso_d;   // Delta(e) table (empty: isotropic)
    int32_t n_cols = 0, max_rows = 0;
    int64_t n_texels = 0;
    std::vector<int32_t> n_rows;
    std::vector<int64_t> col_off;
    std::vector<float> dxy;
    std::vector<int32_t> ord;            // trace order (Morton order of the screen offsets)
    double rho_max = 0;                  // film radius of the last column centre
    std::vector<float> u_of_rho;         // 2 * (kURhoN + 1) floats
    double u_margin = 1.0;               // bound on the table's error, in columns
    // LMFR / LaFR
    double delta = 0, alpha = 0;
    double lf_a = 0, lf_beta = 0;         // LaFR
    std::vector<double> lm_z, lm_cos, lm_sin;   // lm_z: LMFR only
    // device copies
    std::mutex mu;
    std::deque<vafr::LayoutDev> dev;   // stable addresses across push_back
};

namespace vafr {

// ------------------------------------------------------------------ layout
int build_segments(int n_piv, const double* ecc, const double* cpd, Segments* s);
double seg_u(const Segments& s, double e);
double seg_e_of_u(const Segments& s, double u);
double seg_l(const Segments& s, double e);
void film_pitch(const vafr_display& d, double* px, double* py);
// Upload (once per device) and return the tables of the current device.
int layout_device(vafr_layout L, const LayoutDev** out);

// -------------------------------------------------------------------- BVH
// Device node: up to four child boxes, quantised, and four references
// (64 bytes; the traversal is bound by the bytes its lanes load).
//   org  = (origin.x, origin.y, origin.z, scale.z): the node's box corner
//          and the z scale;
//   q0   = (lo.x, hi.x, lo.y, hi.y), q1 = (lo.z, hi.z, scale.x, scale.y):
//          8-bit plane codes, child c in byte c, and the x and y scales;
//          every scale is a power of two, plane = origin + code x scale.
//   ref  = the four child references.
// Every decoded plane, computed as fmaf(code, scale, origin), lies outside
// the child's padded FP32 box (the builder checks each one).
// ref >= 0: internal node index; ref == kEmptyRef: no child (skipped by its
// reference); otherwise a leaf, ~ref = first << 3 | (count-1).
struct alignas(16) BvhNode {
    float4 org;
    uint4 q0, q1;
    int4 ref;
};
static_assert(sizeof(BvhNode) == 64, "quantised 4-wide nodes are 64 bytes");
constexpr int kMaxLeaf = 4;
// Traversal stack: a class of entries per lane in LDS, continued by
// kStackSpill entries per lane in private (scratch) memory.  A node step
// pushes the node's other hit children, so a traversal holds at most the
// sum of (children - 1) over the ancestors of the current node; the binary
// build tree is kept below depth class - 1 and its collapse into 4-wide
// nodes keeps that sum within class + kStackSpill.  The entries past
// min(class, kStackLds) live in scratch (see kStackLds), so only traversals
// holding more than that many entries touch scratch.  The short class keeps
// the scratch part small, the long class admits every supported scene.
constexpr int kStackShort = 24;
constexpr int kStackLong = 32;
constexpr int kStackSpill = 24;
// Of a lane's class + kStackSpill entries, the first min(class, kStackLds)
// live in LDS and the rest in scratch.  20 LDS entries (10 KB per
// 128-thread workgroup) let the Lambert-only kernels (64 VGPRs) keep eight
// waves per SIMD resident where 24 entries allowed 6.5; the deeper entries
// are rarely touched.
constexpr int kStackLds = 20;
// Scenes whose leaf count needs at most this many balanced levels get the
// short class (two levels of slack for the SAH splits).
constexpr int kShortStackLevels = kStackShort - 3;
constexpr int32_t kEmptyRef = INT32_MIN;

struct HostBvh {
    std::vector<BvhNode> nodes;
    std::vector<float4> tris;    // 3 float4 per stored triangle: v0|id, v1, v2
    std::vector<int32_t> order;  // original id of each stored triangle
    int32_t root = kEmptyRef;
    int32_t max_depth = 0;       // binary tree levels below the root
    int32_t wide_depth = 0;      // 4-wide node levels
    int32_t max_stack = 0;       // most stack entries a traversal can hold
    int32_t stack = kStackShort; // traversal stack class (kStackShort or kStackLong)
    float pad = 0.0f;            // absolute padding of every stored box
    float fma_origin_limit = 0;  // origins up to this |component| move a slab plane by <= pad / 8 (fast form)
    int64_t n_leaves = 0;
};

int build_bvh(const float* xyz, int64_t n_verts, const int32_t* tri, int64_t n_tris, HostBvh* out);

}  // namespace vafr

struct vafr_scene_s {
    vafr::HostBvh host;
    int64_t n_tris = 0;
    int device = -1;
    vafr::BvhNode* d_nodes = nullptr;
    float4* d_tris = nullptr;
    int64_t device_bytes = 0;
    double build_ms = 0;
};

namespace vafr {

// ------------------------------------------------------------ trace kernels
enum RayMode : int32_t { kModeVafr = 0, kModeLmfr = 1, kModeFull = 2 };

// Everything one view's rays need; passed by value (kernel argument) or
// stored in a device array for batched launches.
struct TraceView {
    int32_t mode;
    int32_t shade_mode;     // VAFR_SHADE_*
    int64_t n_items;        // work items (padded to whole 8 x 8 tiles for tiled modes)
    // scene
    const BvhNode* nodes;
    const float4* tris;
    int32_t root;
    int32_t stack;          // stack class of the scene (entries per lane)
    float fma_origin_limit; // largest |origin| component for the FMA slab test
    // camera
    float eye[3], right[3], up[3], fwd[3];
    // film geometry (FP64): gaze point on the film and pixel pitch
    double gx, gy, px, py;
    int32_t width, height;
    // VaFR: item k traces texel ord[k] through film offset dxy[k]
    const float2* dxy;
    const int32_t* ord;
    // LMFR / LaFR (dense buffer)
    const double* lm_z;     // LMFR: z per column; NULL for LaFR
    const double2* lm_cs;
    int32_t lm_w, lm_h;
    double lm_L;
    // LaFR kernel (Sec. 4.1 Eq. (15)) at this view's gaze: column abscissa
    // t <= U_ef holds z = t^Fa / (1 - Fa); above it, s = ((t - U_ef) /
    // (1 - U_ef))^(0.7/beta) and 1/z = 1/Z_ef - sin(pi s / 2) (1/Z_ef - 1).
    int32_t lf_on;
    double lf_fa, lf_uef, lf_sexp, lf_zef_inv, lf_k;
    // shading
    float light_dir[3], light_rgb[3], ambient[3], background[3];
    int32_t shadow;
    int32_t bounces;
    uint32_t seed_lo, seed_hi, frame, view;
    // outputs
    float4* out_rgba;
    int32_t* out_id;
    float4* out_p;          // nullable: primary hit point (w = 1) or zeros
    // item list (nullable): the first *item_count entries of item_list are
    // traced, one per thread; n_items bounds the list.
    const int32_t* item_list;
    const int32_t* item_count;
    // Batched path mode in phases (pt_phased = 1): bounces 0 .. kPathFuse of
    // every path run in the traversal launch, and each later bounce b in a
    // queue launch over the compacted list of the paths still alive.  Per
    // path (trace item p) pt_state[4 p ..] holds the next ray's origin |
    // output index, its direction, the throughput | n.l of the last hit and
    // the radiance so far; it is read and written around the traversals, so
    // no path state stays live across them.  pt_list holds two lists of
    // n_items path ids: bounce b reads list b & 1 and appends the paths that
    // continue to list (b + 1) & 1, counted in pt_count[b + 1] (pt_count[0 ..
    // kMaxBounces] is zeroed before the frame).
    float4* pt_state;
    int32_t* pt_list;
    uint32_t* pt_count;
    int32_t pt_phased;
};

// Work items of a view (padded to whole tiles for full-resolution / LMFR).
int64_t trace_items_of(const TraceView& v);
// Traversal workgroup sizes compiled in (one ray per thread).
bool trace_block_ok(int block);
constexpr int kTraceBlockDefault = 128;
// counters != nullptr selects the diagnostic work-counting pass.
int launch_trace(const TraceView& v, hipStream_t stream, unsigned long long* counters = nullptr,
                 int block = kTraceBlockDefault);
// One launch over several views: workgroup b serves the view whose running
// workgroup count block_end[] first exceeds b.
// stack = the largest stack class among the views' scenes; phased: some view
// is a phased path-mode view (TraceView::pt_phased); lambert: every view is
// Lambert-shaded (selects the kernel without the path-tracing code).
int launch_trace_batch(const TraceView* views_dev, const int32_t* block_end_dev, int32_t n_views, int32_t blocks,
                       int block, int stack, bool phased, bool lambert, hipStream_t stream,
                       unsigned long long* counters = nullptr, const int32_t* order = nullptr,
                       uint32_t* cost = nullptr);
// Longest-first dispatch order of a batched traversal launch of `blocks`
// workgroups from the block durations the previous launch recorded in
// cost[] (order: `blocks` entries, one planned permutation per XCD;
// cost[] is cleared as it is read).  trace_plan_ok: whether a launch of
// that size can be planned.
bool trace_plan_ok(int32_t blocks);
// Bounce `bounce` (> kPathFuse) of the phased path-mode views of a batched launch:
// workgroup b serves view vid with qblock_end[vid-1] <= b < qblock_end[vid];
// its thread q traces listed path q while q < pt_count[bounce].
int launch_trace_queue_batch(const TraceView* views_dev, const int32_t* qblock_end_dev, int32_t n_views,
                             int32_t blocks, int stack, int bounce, hipStream_t stream);
const void* trace_queue_batch_kernel(int stack);
constexpr int kQueueBlock = 128;
constexpr int kMaxBounces = 8;
// Bounces 0 .. kPathFuse of a phased path-mode view run in the traversal
// launch, one path per thread; the queue launches take bounce kPathFuse + 1
// on.
constexpr int kPathFuse = 1;
int launch_trace_plan(uint32_t* cost, int32_t* order, int32_t blocks, hipStream_t stream);
const void* trace_plan_kernel();

// ------------------------------------------------------- reconstruction
// One view of the inverse map.  The offset of pixel (x, y)'s centre from the
// gaze point is (x sx + cx, y sy + cy): film units for VaFR, pixels for LMFR.
struct ReconView {
    int32_t mode;       // kModeVafr or kModeLmfr
    int32_t width, height;
    int32_t n_cols;     // VaFR columns / LMFR buffer width
    int32_t lm_h;       // LMFR buffer height
    float sx, sy, cx, cy;
    // VaFR
    float rho_scale;    // kURhoN / rho_max
    const float2* u_of_rho;
    const int2* col;    // (n_rows, col_off)
    // LMFR / LaFR
    double lm_cx, lm_cy; // pixel (x, y) centre minus the gaze point = (x + lm_cx, y + lm_cy), FP64
    float inv_L;        // ln 2 / L (the kernel uses log2)
    float alpha;
    // LaFR (Sec. 4.1 Eq. (15)): z <= Z_ef gives (z (1 - Fa))^(1/Fa); above,
    // Za = (1/z - 1/Z_ef) / (1/Z_ef - 1) and
    // ((2 acos Za - pi) / pi)^(beta/0.7) (1 - U_ef) + U_ef.
    int32_t lf_on;
    float lf_zef, lf_fa1, lf_inv_fa, lf_k, lf_uef, lf_bexp;
    float lf_half_inv_lnl;  // 1 / (2 ln L)
    double lf_inv_r2;       // 1 / R^2, R = e^(ln L) the farthest corner's distance in pixels
    const float4* lp;
    uint32_t lp_bytes;  // < 2^32
    float4* img;
    // batched frames: a second VaFR view with the same layout, gaze and
    // display (the other eye), reconstructed in the same pass; or null
    const float4* lp2;
    float4* img2;
};

// Reconstruction workgroups have kReconThreads threads (4 waves); `rows` is
// the number of display rows each thread writes, so a tile is 64 x 4 rows.
constexpr int kReconThreads = 256;
bool recon_rows_ok(int rows);
constexpr int kReconRowsDefault = 8;        // per-view calls
constexpr int kBatchReconRowsDefault = 4;   // batches: binocular pairs fit 64 VGPRs at 4 rows, not at 8
int64_t recon_blocks_of(const ReconView& v, int rows);
int launch_reconstruct(const ReconView& v, hipStream_t stream, int rows = kReconRowsDefault);
int launch_reconstruct_batch(const ReconView* views_dev, const int32_t* block_end_dev, int32_t n_views,
                             int32_t blocks, int rows, hipStream_t stream);

// Binocular reprojection: clear the per-texel keys and splat the left hit
// points into the right eye's LP cells.
// Binocular reprojection into the right eye (per texel of a VaFR layout) by
// forward grid warping: clears the texel keys and the hole count, warps the
// grid triangles of the left hit points (depth-ordered atomic minimum per
// covered right texel), then writes each covered texel's interpolated
// colour and hit id into the right buffers and lists the trace-order items
// of the texels no triangle covered.
struct RepBuffers {
    const float4* points;         // left hit points (w = 1) or zeros
    unsigned long long* key;      // per right texel: depth bits << 32 | triangle id
    const float4* src_rgba;       // left LP buffer
    const int32_t* src_id;        // nullable
    float4* out_rgba;             // right LP buffer
    int32_t* out_id;              // nullable
    int32_t* list;                // hole items, trace order within a workgroup
    int32_t* count;               // number of listed holes
};
int launch_rep(const LayoutDev& ld, const vafr_layout_s& L, double gx, double gy, const vafr_camera& right,
               const RepBuffers& b, hipStream_t stream);

// LP anti-aliasing over all texels of a VaFR layout (col: per-column rows
// and first texel on the device).
constexpr int kTexelBlock = 256;   // texels per workgroup of per-texel kernels
int launch_fxaa(const int2* col_dev, const int32_t* blk_col_dev, int32_t n_cols, int64_t n_texels, const float* in,
                float* out, hipStream_t stream);

// vafr_shade_lp_rep on a given workspace (validation included); the
// allocation-free entry point passes its static scratch array.
int shade_lp_rep_ws(vafr_scene scene, const vafr_camera* cam_left, const vafr_camera* cam_right, vafr_gaze gaze,
                    const vafr_shading* sh, vafr_layout L, float* lp_left, float* lp_right, int32_t* hit_left,
                    int32_t* hit_right, void* ws, int64_t ws_bytes, hipStream_t stream, hipStream_t right_stream);
// Whether the layout's tables are already on the current device (no upload).
int layout_resident(vafr_layout L, bool* resident);

// Per-view descriptors from the public arguments (validated; uploads the
// layout tables to the current device on first use).
int make_trace_view(int kind, vafr_scene scene, const vafr_camera* cam, vafr_gaze gaze, const vafr_shading* sh,
                    vafr_layout L, const vafr_display* disp, float* out_rgba, int32_t* hit, TraceView* v);
int make_recon_view(vafr_layout L, vafr_gaze gaze, const float* lp, float* img, ReconView* r);

// Kernel entry points of the batched launches (for graph nodes); their
// parameters are (views, block_end, n_views[, counters]).
const void* trace_batch_kernel(int block, int stack, bool phased, bool lambert);
const void* recon_batch_kernel(int rows);

// common validation helpers
int check_camera(const vafr_camera* c);
int check_shading(const vafr_shading* s);
int check_gaze(vafr_gaze g);

}  // namespace vafr
