// C ABI entry points: argument validation, handle management and the
// per-frame launches.  Host arithmetic on the film geometry is FP64.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "vafr_internal.h"

namespace vafr {

static thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(VAFR_E_HIP, "%s failed: %s", what, hipGetErrorString(e));
}

int check_camera(const vafr_camera* c) {
    if (!c) return fail(VAFR_E_ARG, "camera is NULL");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(c->eye[k]) || !std::isfinite(c->right[k]) || !std::isfinite(c->up[k]) ||
            !std::isfinite(c->forward[k]))
            return fail(VAFR_E_ARG, "camera has a non-finite component");
    return VAFR_OK;
}

int check_shading(const vafr_shading* s) {
    if (!s) return fail(VAFR_E_ARG, "shading is NULL");
    if (s->mode != VAFR_SHADE_LAMBERT && s->mode != VAFR_SHADE_PATH) return fail(VAFR_E_ARG, "unknown shading mode");
    if (s->shadow_rays != 0 && s->shadow_rays != 1) return fail(VAFR_E_ARG, "shadow_rays must be 0 or 1");
    if (s->mode == VAFR_SHADE_PATH && (s->bounces < 0 || s->bounces > 8))
        return fail(VAFR_E_ARG, "bounces must be in [0, 8]");
    double l2 = 0;
    for (int k = 0; k < 3; ++k) {
        if (!std::isfinite(s->light_dir[k]) || !std::isfinite(s->light_rgb[k]) || !std::isfinite(s->ambient[k]) ||
            !std::isfinite(s->background[k]))
            return fail(VAFR_E_ARG, "shading has a non-finite component");
    }
    l2 = ((double)s->light_dir[0] * s->light_dir[0] + (double)s->light_dir[1] * s->light_dir[1]) +
         (double)s->light_dir[2] * s->light_dir[2];
    if (!(l2 >= 1e-30) || !std::isfinite(l2)) return fail(VAFR_E_ARG, "light_dir must be a non-zero vector");
    return VAFR_OK;
}

int check_gaze(vafr_gaze g) {
    if (!std::isfinite(g.x_px) || !std::isfinite(g.y_px)) return fail(VAFR_E_ARG, "gaze is not finite");
    if (std::fabs(g.x_px) > 1e7 || std::fabs(g.y_px) > 1e7) return fail(VAFR_E_ARG, "gaze is out of range");
    return VAFR_OK;
}

static int current_device(int* dev) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return fail(VAFR_E_HIP, "no HIP device available");
    VAFR_HIP(hipGetDevice(dev));
    return VAFR_OK;
}

static int scene_into_view(vafr_scene s, TraceView* v) {
    if (!s) return fail(VAFR_E_ARG, "scene is NULL");
    int dev;
    if (int rc = current_device(&dev)) return rc;
    if (s->n_tris > 0 && s->device != dev)
        return fail(VAFR_E_ARG, "scene lives on device %d, current device is %d", s->device, dev);
    v->nodes = s->d_nodes;
    v->tris = s->d_tris;
    v->root = s->host.root;
    v->stack = s->host.stack;
    v->fma_origin_limit = s->host.fma_origin_limit;
    return VAFR_OK;
}

static void fill_view_common(TraceView& v, const vafr_camera* cam, const vafr_shading* sh) {
    std::memcpy(v.eye, cam->eye, sizeof(v.eye));
    std::memcpy(v.right, cam->right, sizeof(v.right));
    std::memcpy(v.up, cam->up, sizeof(v.up));
    std::memcpy(v.fwd, cam->forward, sizeof(v.fwd));
    // the light direction is normalised here: FP64 from the FP32 input,
    // squares summed as (x x + y y) + z z, rounded once to FP32
    const double lx = sh->light_dir[0], ly = sh->light_dir[1], lz = sh->light_dir[2];
    const double len = std::sqrt((lx * lx + ly * ly) + lz * lz);
    v.light_dir[0] = (float)(lx / len);
    v.light_dir[1] = (float)(ly / len);
    v.light_dir[2] = (float)(lz / len);
    std::memcpy(v.light_rgb, sh->light_rgb, sizeof(v.light_rgb));
    std::memcpy(v.ambient, sh->ambient, sizeof(v.ambient));
    std::memcpy(v.background, sh->background, sizeof(v.background));
    v.shade_mode = sh->mode;
    v.shadow = sh->shadow_rays;
    v.bounces = sh->mode == VAFR_SHADE_PATH ? sh->bounces : 0;
    v.seed_lo = (uint32_t)sh->seed;
    v.seed_hi = (uint32_t)(sh->seed >> 32);
    v.frame = sh->frame;
    v.view = sh->view;
}

// Gaze point on the film plane (unit focal length).
static void gaze_film(const vafr_layout_s* L, vafr_gaze g, double* gx, double* gy) {
    *gx = (g.x_px - 0.5 * L->disp.width) * L->px;
    *gy = (g.y_px - 0.5 * L->disp.height) * L->py;
}

// LMFR's L (Sec. 3.1, Eq. (1)): log of the longest pixel distance from the
// gaze point to a screen corner.
static double lmfr_log_extent(const vafr_layout_s* L, vafr_gaze g) {
    const double cx[4] = {0.0, (double)L->disp.width, 0.0, (double)L->disp.width};
    const double cy[4] = {0.0, 0.0, (double)L->disp.height, (double)L->disp.height};
    double best = 0.0;
    for (int c = 0; c < 4; ++c) {
        const double dx = cx[c] - g.x_px, dy = cy[c] - g.y_px;
        const double d = std::sqrt(dx * dx + dy * dy);
        if (d > best) best = d;
    }
    return std::log(best);
}

// LaFR kernel constants at one gaze (Sec. 4.1 Eq. (15)): Z_ef = z(4.89 deg)
// with z(e) = ln(tan e / c_r) / ln L and c_r the vertical film pitch of a
// pixel; Fa = 1 - log_{Z_ef}((alpha Z_ef)^(1-a) / (1-a)); U_ef =
// (Z_ef (1 - Fa))^(1/Fa).  FP64.
struct LafrConsts {
    double lnL, zef, fa, uef;
};

static int lafr_consts(const vafr_layout_s* L, vafr_gaze g, LafrConsts* c) {
    constexpr double kFovealDeg = 4.89;
    c->lnL = lmfr_log_extent(L, g);
    if (!(c->lnL > 0.0)) return fail(VAFR_E_ARG, "display too small for the LaFR map");
    c->zef = std::log(std::tan(kFovealDeg * M_PI / 180.0) / L->py) / c->lnL;
    if (!(c->zef > 0.0 && c->zef < 1.0))
        return fail(VAFR_E_ARG, "LaFR foveal boundary outside the screen at this gaze (Z_ef = %g)", c->zef);
    const double a = L->lf_a;
    c->fa = 1.0 - std::log(std::pow(L->alpha * c->zef, 1.0 - a) / (1.0 - a)) / std::log(c->zef);
    if (!(c->fa > 0.0 && c->fa < 1.0)) return fail(VAFR_E_ARG, "LaFR kernel undefined at this gaze (Fa = %g)", c->fa);
    c->uef = std::pow(c->zef * (1.0 - c->fa), 1.0 / c->fa);
    return VAFR_OK;
}

// kind: VAFR_LAYOUT_VAFR / VAFR_LAYOUT_LMFR / VAFR_LAYOUT_LAFR (layout
// given) or -1 for the full-resolution view of `disp`.
int make_trace_view(int kind, vafr_scene scene, const vafr_camera* cam, vafr_gaze gaze, const vafr_shading* sh,
                    vafr_layout L, const vafr_display* disp, float* out_rgba, int32_t* hit, TraceView* out) {
    if (int rc = check_camera(cam)) return rc;
    if (int rc = check_shading(sh)) return rc;
    TraceView v;
    std::memset(&v, 0, sizeof(v));
    if (kind < 0) {
        if (!disp) return fail(VAFR_E_ARG, "display is NULL");
        if (disp->width <= 0 || disp->height <= 0 || disp->width > 65536 || disp->height > 65536)
            return fail(VAFR_E_ARG, "display size out of range");
        if (!(disp->fov_x_deg > 0.0 && disp->fov_x_deg < 180.0) || !(disp->fov_y_deg > 0.0 && disp->fov_y_deg < 180.0))
            return fail(VAFR_E_ARG, "field of view must lie in (0, 180) degrees");
    } else {
        if (!L) return fail(VAFR_E_ARG, "layout is NULL");
        if (L->kind != kind)
            return fail(VAFR_E_ARG, kind == VAFR_LAYOUT_VAFR   ? "vafr_shade_lp needs a VaFR layout"
                                    : kind == VAFR_LAYOUT_LMFR ? "lmfr_shade_lp needs an LMFR layout"
                                                               : "lafr_shade_lp needs a LaFR layout");
        if (int rc = check_gaze(gaze)) return rc;
    }
    if (int rc = scene_into_view(scene, &v)) return rc;
    fill_view_common(v, cam, sh);
    if (kind < 0) {
        v.mode = kModeFull;
        v.width = disp->width;
        v.height = disp->height;
        film_pitch(*disp, &v.px, &v.py);
    } else {
        const LayoutDev* ld;
        if (int rc = layout_device(L, &ld)) return rc;
        gaze_film(L, gaze, &v.gx, &v.gy);
        v.px = L->px;
        v.py = L->py;
        v.width = L->disp.width;
        v.height = L->disp.height;
        if (kind == VAFR_LAYOUT_VAFR) {
            v.mode = kModeVafr;
            v.n_items = L->n_texels;
            v.dxy = ld->dxy;
            v.ord = ld->ord;
        } else {
            v.mode = kModeLmfr;
            v.lm_z = ld->lm_z;
            v.lm_cs = ld->lm_cs;
            v.lm_w = L->n_cols;
            v.lm_h = L->max_rows;
            v.lm_L = lmfr_log_extent(L, gaze);
            if (!(v.lm_L > 0.0)) return fail(VAFR_E_ARG, "display too small for the LMFR map");
            if (kind == VAFR_LAYOUT_LAFR) {
                LafrConsts c;
                if (int rc = lafr_consts(L, gaze, &c)) return rc;
                v.lf_on = 1;
                v.lf_fa = c.fa;
                v.lf_uef = c.uef;
                v.lf_sexp = 0.7 / L->lf_beta;
                v.lf_zef_inv = 1.0 / c.zef;
                v.lf_k = 1.0 / c.zef - 1.0;
            }
        }
    }
    v.out_rgba = reinterpret_cast<float4*>(out_rgba);
    v.out_id = hit;
    v.n_items = trace_items_of(v);
    *out = v;
    return VAFR_OK;
}

int make_recon_view(vafr_layout L, vafr_gaze gaze, const float* lp, float* img, ReconView* out) {
    if (!L) return fail(VAFR_E_ARG, "layout is NULL");
    if (int rc = check_gaze(gaze)) return rc;
    if (!lp || !img) return fail(VAFR_E_ARG, "NULL buffer");
    int dev;
    if (int rc = current_device(&dev)) return rc;
    ReconView r;
    std::memset(&r, 0, sizeof(r));
    r.width = L->disp.width;
    r.height = L->disp.height;
    r.n_cols = L->n_cols;
    r.lp = reinterpret_cast<const float4*>(lp);
    r.img = reinterpret_cast<float4*>(img);
    if (L->n_texels * 16 >= ((int64_t)1 << 32))
        return fail(VAFR_E_UNSUPPORTED, "LP buffers of 2^28 texels or more are not supported");
    r.lp_bytes = (uint32_t)(L->n_texels * 16);
    if (L->kind == VAFR_LAYOUT_VAFR) {
        const LayoutDev* ld;
        if (int rc = layout_device(L, &ld)) return rc;
        double gx, gy;
        gaze_film(L, gaze, &gx, &gy);
        r.mode = kModeVafr;
        r.sx = (float)L->px;
        r.sy = (float)L->py;
        r.cx = (float)((0.5 - 0.5 * L->disp.width) * L->px - gx);
        r.cy = (float)((0.5 - 0.5 * L->disp.height) * L->py - gy);
        r.rho_scale = (float)(kURhoN / L->rho_max);
        r.u_of_rho = ld->u_of_rho;
        r.col = ld->col;
    } else {
        const double Lg = lmfr_log_extent(L, gaze);
        if (!(Lg > 0.0)) return fail(VAFR_E_ARG, "display too small for the LMFR map");
        r.mode = kModeLmfr;
        r.lm_h = L->max_rows;
        r.sx = r.sy = 1.0f;
        r.cx = (float)(0.5 - gaze.x_px);
        r.cy = (float)(0.5 - gaze.y_px);
        r.lm_cx = 0.5 - gaze.x_px;
        r.lm_cy = 0.5 - gaze.y_px;
        r.inv_L = (float)(M_LN2 / Lg);
        r.alpha = (float)L->alpha;
        if (L->kind == VAFR_LAYOUT_LAFR) {
            LafrConsts c;
            if (int rc = lafr_consts(L, gaze, &c)) return rc;
            r.lf_on = 1;
            r.lf_zef = (float)c.zef;
            r.lf_fa1 = (float)(1.0 - c.fa);
            r.lf_inv_fa = (float)(1.0 / c.fa);
            r.lf_k = (float)(1.0 / c.zef - 1.0);
            r.lf_uef = (float)c.uef;
            r.lf_bexp = (float)(L->lf_beta / 0.7);
            r.lf_half_inv_lnl = (float)(0.5 / c.lnL);
            r.lf_inv_r2 = std::exp(-2.0 * c.lnL);
        }
    }
    *out = r;
    return VAFR_OK;
}

}  // namespace vafr

using namespace vafr;

extern "C" const char* vafr_last_error(void) { return g_err; }

extern "C" int vafr_abi_version(void) { return 2; }

extern "C" int vafr_scene_create(const float* xyz, int64_t n_verts, const int32_t* tri, int64_t n_tris,
                                 vafr_scene* out) {
    if (!out) return fail(VAFR_E_ARG, "out is NULL");
    *out = nullptr;
    if (n_tris < 0 || n_verts < 0) return fail(VAFR_E_ARG, "negative count");
    if (n_tris >= ((int64_t)1 << 27)) return fail(VAFR_E_UNSUPPORTED, "at most 2^27 - 1 triangles");
    if (n_tris > 0 && (!xyz || !tri)) return fail(VAFR_E_ARG, "NULL scene arrays");
    vafr_scene s = new (std::nothrow) vafr_scene_s;
    if (!s) return fail(VAFR_E_OOM, "scene allocation failed");
    s->n_tris = n_tris;
    const auto t0 = std::chrono::steady_clock::now();
    int rc;
    try {
        rc = build_bvh(xyz, n_verts, tri, n_tris, &s->host);
    } catch (const std::bad_alloc&) {
        rc = fail(VAFR_E_OOM, "BVH build ran out of host memory");
    }
    s->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rc) { delete s; return rc; }
    if (s->host.max_depth > s->host.stack - 1 || s->host.max_stack > s->host.stack + kStackSpill) {
        delete s;
        return fail(VAFR_E_UNSUPPORTED, "BVH depth exceeds the traversal stack");
    }
    int n_dev = 0;
    if (n_tris > 0 && hipGetDeviceCount(&n_dev) == hipSuccess && n_dev > 0) {
        auto cleanup = [&](int code) { vafr_scene_destroy(s); return code; };
        if (hipGetDevice(&s->device) != hipSuccess) return cleanup(fail(VAFR_E_HIP, "hipGetDevice failed"));
        const size_t nb = sizeof(BvhNode) * s->host.nodes.size();
        const size_t tb = sizeof(float4) * s->host.tris.size();
        if (nb && hipMalloc(&s->d_nodes, nb) != hipSuccess) return cleanup(fail(VAFR_E_OOM, "hipMalloc of BVH nodes"));
        if (hipMalloc(&s->d_tris, tb) != hipSuccess) return cleanup(fail(VAFR_E_OOM, "hipMalloc of triangles"));
        if (nb && hipMemcpy(s->d_nodes, s->host.nodes.data(), nb, hipMemcpyHostToDevice) != hipSuccess)
            return cleanup(fail(VAFR_E_HIP, "upload of BVH nodes failed"));
        if (hipMemcpy(s->d_tris, s->host.tris.data(), tb, hipMemcpyHostToDevice) != hipSuccess)
            return cleanup(fail(VAFR_E_HIP, "upload of triangles failed"));
        s->device_bytes = (int64_t)(nb + tb);
    }
    *out = s;
    return VAFR_OK;
}

extern "C" int vafr_scene_get_info(vafr_scene s, vafr_scene_info* out) {
    if (!s || !out) return fail(VAFR_E_ARG, "NULL argument");
    out->n_tris = s->n_tris;
    out->n_nodes = (int64_t)s->host.nodes.size();
    out->n_leaves = s->host.n_leaves;
    out->max_depth = s->host.max_depth;
    out->on_device = s->d_tris != nullptr;
    out->device_bytes = s->device_bytes;
    out->build_ms = s->build_ms;
    out->stack_entries = s->host.stack;
    out->max_stack = s->host.max_stack;
    return VAFR_OK;
}

extern "C" int vafr_scene_export(vafr_scene s, float* nodes, int32_t* tri_order) {
    if (!s) return fail(VAFR_E_ARG, "scene is NULL");
    if (nodes && !s->host.nodes.empty())
        std::memcpy(nodes, s->host.nodes.data(), sizeof(BvhNode) * s->host.nodes.size());
    if (tri_order && !s->host.order.empty())
        std::memcpy(tri_order, s->host.order.data(), sizeof(int32_t) * s->host.order.size());
    return VAFR_OK;
}

extern "C" void vafr_scene_destroy(vafr_scene s) {
    if (!s) return;
    if (s->device >= 0) {
        int cur = -1;
        const bool have = hipGetDevice(&cur) == hipSuccess;
        if (hipSetDevice(s->device) == hipSuccess) {
            (void)hipFree(s->d_nodes);
            (void)hipFree(s->d_tris);
        }
        if (have) (void)hipSetDevice(cur);
    }
    delete s;
}

extern "C" int vafr_shade_lp(vafr_scene scene, const vafr_camera* cam, vafr_gaze gaze, const vafr_shading* sh,
                             vafr_layout L, float* lp, int32_t* hit, hipStream_t stream) {
    if (!lp) return fail(VAFR_E_ARG, "lp_rgba_dev is NULL");
    TraceView v;
    if (int rc = make_trace_view(VAFR_LAYOUT_VAFR, scene, cam, gaze, sh, L, nullptr, lp, hit, &v)) return rc;
    return launch_trace(v, stream);
}

extern "C" int lmfr_shade_lp(vafr_scene scene, const vafr_camera* cam, vafr_gaze gaze, const vafr_shading* sh,
                             vafr_layout L, float* lp, int32_t* hit, hipStream_t stream) {
    if (!lp) return fail(VAFR_E_ARG, "lp_rgba_dev is NULL");
    TraceView v;
    if (int rc = make_trace_view(VAFR_LAYOUT_LMFR, scene, cam, gaze, sh, L, nullptr, lp, hit, &v)) return rc;
    return launch_trace(v, stream);
}

extern "C" int lafr_shade_lp(vafr_scene scene, const vafr_camera* cam, vafr_gaze gaze, const vafr_shading* sh,
                             vafr_layout L, float* lp, int32_t* hit, hipStream_t stream) {
    if (!lp) return fail(VAFR_E_ARG, "lp_rgba_dev is NULL");
    TraceView v;
    if (int rc = make_trace_view(VAFR_LAYOUT_LAFR, scene, cam, gaze, sh, L, nullptr, lp, hit, &v)) return rc;
    return launch_trace(v, stream);
}

static int reconstruct_kind(int kind, vafr_layout L, vafr_gaze gaze, const float* lp, float* img, hipStream_t stream) {
    if (!L) return fail(VAFR_E_ARG, "layout is NULL");
    if (L->kind != kind)
        return fail(VAFR_E_ARG, kind == VAFR_LAYOUT_VAFR   ? "vafr_reconstruct needs a VaFR layout"
                                : kind == VAFR_LAYOUT_LMFR ? "lmfr_reconstruct needs an LMFR layout"
                                                           : "lafr_reconstruct needs a LaFR layout");
    ReconView r;
    if (int rc = make_recon_view(L, gaze, lp, img, &r)) return rc;
    return launch_reconstruct(r, stream);
}

extern "C" int vafr_reconstruct(vafr_layout L, vafr_gaze gaze, const float* lp, float* img, hipStream_t stream) {
    return reconstruct_kind(VAFR_LAYOUT_VAFR, L, gaze, lp, img, stream);
}

extern "C" int lmfr_reconstruct(vafr_layout L, vafr_gaze gaze, const float* lp, float* img, hipStream_t stream) {
    return reconstruct_kind(VAFR_LAYOUT_LMFR, L, gaze, lp, img, stream);
}

extern "C" int lafr_reconstruct(vafr_layout L, vafr_gaze gaze, const float* lp, float* img, hipStream_t stream) {
    return reconstruct_kind(VAFR_LAYOUT_LAFR, L, gaze, lp, img, stream);
}

extern "C" int vafr_rep_workspace_bytes(vafr_layout L, int64_t* bytes) {
    if (!L || !bytes) return fail(VAFR_E_ARG, "NULL argument");
    if (L->kind != VAFR_LAYOUT_VAFR) return fail(VAFR_E_UNSUPPORTED, "reprojection needs a VaFR layout");
    // hit points, cell keys, hole list, hole count (padded to 16 bytes)
    *bytes = L->n_texels * (int64_t)(sizeof(float4) + sizeof(unsigned long long) + sizeof(int32_t)) + 16;
    return VAFR_OK;
}

namespace vafr {

int shade_lp_rep_ws(vafr_scene scene, const vafr_camera* cam_left, const vafr_camera* cam_right, vafr_gaze gaze,
                    const vafr_shading* sh, vafr_layout L, float* lp_left, float* lp_right, int32_t* hit_left,
                    int32_t* hit_right, void* ws, int64_t ws_bytes, hipStream_t stream, hipStream_t right_stream) {
    int64_t need;
    if (int rc = vafr_rep_workspace_bytes(L, &need)) return rc;
    if (!lp_left || !lp_right) return fail(VAFR_E_ARG, "LP buffer is NULL");
    if (!ws || ws_bytes < need)
        return fail(VAFR_E_ARG, "workspace of %lld bytes needed, %lld given", (long long)need, (long long)ws_bytes);
    if (reinterpret_cast<uintptr_t>(ws) % 16) return fail(VAFR_E_ARG, "workspace is not 16-byte aligned");
    {
        // the right eye reads the left buffers and the workspace while it
        // writes its own: none of them may overlap
        const uintptr_t lb = (uintptr_t)L->n_texels * 16u, ib = (uintptr_t)L->n_texels * 4u;
        const struct { const void* p; uintptr_t n; } span[5] = {
            {lp_left, lb}, {lp_right, lb}, {ws, (uintptr_t)need}, {hit_left, hit_left ? ib : 0},
            {hit_right, hit_right ? ib : 0}};
        for (int a = 0; a < 5; ++a)
            for (int b = a + 1; b < 5; ++b) {
                const uintptr_t pa = reinterpret_cast<uintptr_t>(span[a].p), pb = reinterpret_cast<uintptr_t>(span[b].p);
                if (span[a].n && span[b].n && pa < pb + span[b].n && pb < pa + span[a].n)
                    return fail(VAFR_E_ARG, "LP buffers, hit-id buffers and workspace must not overlap");
            }
    }
    if (int rc = check_camera(cam_right)) return rc;
    TraceView left, right;
    if (int rc = make_trace_view(VAFR_LAYOUT_VAFR, scene, cam_left, gaze, sh, L, nullptr, lp_left, hit_left, &left))
        return rc;
    if (int rc = make_trace_view(VAFR_LAYOUT_VAFR, scene, cam_right, gaze, sh, L, nullptr, lp_right, hit_right, &right))
        return rc;
    const int64_t n = L->n_texels;
    RepBuffers rb;
    rb.points = reinterpret_cast<float4*>(ws);
    rb.key = reinterpret_cast<unsigned long long*>(reinterpret_cast<float4*>(ws) + n);
    rb.list = reinterpret_cast<int32_t*>(rb.key + n);
    rb.count = rb.list + n;
    rb.src_rgba = reinterpret_cast<const float4*>(lp_left);
    rb.src_id = hit_left;
    rb.out_rgba = reinterpret_cast<float4*>(lp_right);
    rb.out_id = hit_right;
    left.out_p = reinterpret_cast<float4*>(ws);
    right.item_list = rb.list;
    right.item_count = rb.count;
    const LayoutDev* ld;
    if (int rc = layout_device(L, &ld)) return rc;
    if (int rc = launch_trace(left, stream)) return rc;
    double gx, gy;
    gaze_film(L, gaze, &gx, &gy);
    if (int rc = launch_rep(*ld, *L, gx, gy, *cam_right, rb, stream)) return rc;
    if (!right_stream || right_stream == stream) return launch_trace(right, stream);
    // the hole pass on right_stream, after the warp on stream (an event's
    // state is captured by the wait, so it can be destroyed at once)
    hipEvent_t ev;
    VAFR_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ev, stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(right_stream, ev, 0);
    (void)hipEventDestroy(ev);
    VAFR_HIP(e);
    return launch_trace(right, right_stream);
}

}  // namespace vafr

extern "C" int vafr_shade_lp_rep(vafr_scene scene, const vafr_camera* cam_left, const vafr_camera* cam_right,
                                 vafr_gaze gaze, const vafr_shading* sh, vafr_layout L, float* lp_left,
                                 float* lp_right, int32_t* hit_left, int32_t* hit_right, void* ws, int64_t ws_bytes,
                                 hipStream_t stream, hipStream_t right_stream) {
    return shade_lp_rep_ws(scene, cam_left, cam_right, gaze, sh, L, lp_left, lp_right, hit_left, hit_right, ws,
                           ws_bytes, stream, right_stream);
}

extern "C" int vafr_fxaa_lp(vafr_layout L, const float* in, float* out, hipStream_t stream) {
    if (!L) return fail(VAFR_E_ARG, "layout is NULL");
    if (L->kind != VAFR_LAYOUT_VAFR) return fail(VAFR_E_UNSUPPORTED, "LP anti-aliasing needs a VaFR layout");
    if (!in || !out) return fail(VAFR_E_ARG, "LP buffer is NULL");
    const uintptr_t a = reinterpret_cast<uintptr_t>(in), b = reinterpret_cast<uintptr_t>(out);
    const uintptr_t bytes = (uintptr_t)L->n_texels * 16u;
    if (a < b + bytes && b < a + bytes) return fail(VAFR_E_ARG, "input and output LP buffers overlap");
    const LayoutDev* ld;
    if (int rc = layout_device(L, &ld)) return rc;
    return launch_fxaa(ld->col, ld->blk_col, L->n_cols, L->n_texels, in, out, stream);
}

extern "C" int full_shade(vafr_scene scene, const vafr_camera* cam, const vafr_display* d, const vafr_shading* sh,
                          float* img, int32_t* hit, hipStream_t stream) {
    if (!img) return fail(VAFR_E_ARG, "img_rgba_dev is NULL");
    TraceView v;
    if (int rc = make_trace_view(-1, scene, cam, vafr_gaze{0.0, 0.0}, sh, nullptr, d, img, hit, &v)) return rc;
    return launch_trace(v, stream);
}

extern "C" int vafr_count_work(vafr_scene scene, const vafr_camera* cam, vafr_gaze gaze, const vafr_shading* sh,
                               vafr_layout L, unsigned long long* counters_dev, hipStream_t stream) {
    if (!L) return fail(VAFR_E_ARG, "layout is NULL");
    if (!counters_dev) return fail(VAFR_E_ARG, "counters_dev is NULL");
    TraceView v;
    if (int rc = make_trace_view(L->kind, scene, cam, gaze, sh, L, nullptr, nullptr, nullptr, &v)) return rc;
    return launch_trace(v, stream, counters_dev);
}
