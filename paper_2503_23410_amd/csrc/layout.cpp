// Host side of the LP layouts: FP64 acuity segments, the VaFR constant-size
// LP buffer (Sec. 3.2.1-3.2.3, Sec. 3.3) and the LMFR / LaFR comparison
// buffers (Sec. 3.1 Eq. (1), Sec. 4.1 Eq. (14), Eq. (15)), plus their
// per-device upload.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "vafr_internal.h"

namespace vafr {

static constexpr double kDeg = M_PI / 180.0;

// Pivots (e_k, f_k) -> linear MAR per segment (Sec. 3.3): omega(e_k) = 1/f_k,
// omega(e_{k+1}) = 1/f_{k+1}.  u(0) = 0 and u is continuous at the pivots,
// which fixes the constants c_k of Eq. (12).
int build_segments(int n_piv, const double* ecc, const double* cpd, Segments* s) {
    if (n_piv < 2 || n_piv > kMaxSeg + 1) return fail(VAFR_E_ARG, "n_pivots must be in [2, %d]", kMaxSeg + 1);
    if (!ecc || !cpd) return fail(VAFR_E_ARG, "acuity arrays are NULL");
    if (ecc[0] != 0.0) return fail(VAFR_E_ARG, "first pivot eccentricity must be 0");
    for (int k = 0; k < n_piv; ++k) {
        if (!std::isfinite(ecc[k]) || !std::isfinite(cpd[k]) || !(cpd[k] > 0.0))
            return fail(VAFR_E_ARG, "pivot %d: acuity must be finite and > 0", k);
        if (k && !(ecc[k] > ecc[k - 1])) return fail(VAFR_E_ARG, "pivot eccentricities must increase strictly");
    }
    Segments r;
    r.n = n_piv - 1;
    for (int k = 0; k < n_piv; ++k) r.e[k] = ecc[k];
    for (int k = 0; k < r.n; ++k) {
        const double mar0 = 1.0 / cpd[k], mar1 = 1.0 / cpd[k + 1];
        r.m[k] = (mar1 - mar0) / (ecc[k + 1] - ecc[k]);
        r.b[k] = mar0 - r.m[k] * ecc[k];
    }
    auto raw = [&](int k, double e) {
        return r.m[k] == 0.0 ? 2.0 * e / r.b[k] : 2.0 * std::log(r.m[k] * e + r.b[k]) / r.m[k];
    };
    r.u[0] = 0.0;
    for (int k = 0; k < r.n; ++k) {
        r.c[k] = r.u[k] - raw(k, r.e[k]);
        r.u[k + 1] = raw(k, r.e[k + 1]) + r.c[k];
    }
    *s = r;
    return VAFR_OK;
}

// Delta(e) of Eq. (19): linear between the table points, constant outside.
static double aniso_delta(const vafr_layout_s& L, double e) {
    const int n = (int)L.aniso_e.size();
    if (n == 0) return 1.0;
    if (e <= L.aniso_e[0]) return L.aniso_d[0];
    for (int k = 0; k + 1 < n; ++k)
        if (e < L.aniso_e[k + 1]) {
            const double t = (e - L.aniso_e[k]) / (L.aniso_e[k + 1] - L.aniso_e[k]);
            return L.aniso_d[k] + t * (L.aniso_d[k + 1] - L.aniso_d[k]);
        }
    return L.aniso_d[n - 1];
}

static int seg_index_e(const Segments& s, double e) {
    int k = 0;
    while (k + 1 < s.n && e >= s.e[k + 1]) ++k;
    return k;
}

static int seg_index_u(const Segments& s, double u) {
    int k = 0;
    while (k + 1 < s.n && u >= s.u[k + 1]) ++k;
    return k;
}

// Eq. (5) on the segment holding e; the last segment extends past e_max.
double seg_u(const Segments& s, double e) {
    const int k = seg_index_e(s, e);
    if (s.m[k] == 0.0) return 2.0 * e / s.b[k] + s.c[k];
    return 2.0 * std::log(s.m[k] * e + s.b[k]) / s.m[k] + s.c[k];
}

// Eq. (10) on the segment holding u.
double seg_e_of_u(const Segments& s, double u) {
    const int k = seg_index_u(s, u);
    if (s.m[k] == 0.0) return (u - s.c[k]) * s.b[k] * 0.5;
    return (std::exp((u - s.c[k]) * s.m[k] * 0.5) - s.b[k]) / s.m[k];
}

// Eq. (9): l(e) = 360 sin(2e) / omega(e).
double seg_l(const Segments& s, double e) {
    const int k = seg_index_e(s, e);
    return 360.0 * std::sin(2.0 * e * kDeg) / (s.m[k] * e + s.b[k]);
}

// Film plane at unit focal length; a pixel spans 2 tan(fov/2) / size.
void film_pitch(const vafr_display& d, double* px, double* py) {
    *px = 2.0 * std::tan(0.5 * d.fov_x_deg * kDeg) / d.width;
    *py = 2.0 * std::tan(0.5 * d.fov_y_deg * kDeg) / d.height;
}

static int check_display(const vafr_display* d) {
    if (!d) return fail(VAFR_E_ARG, "display is NULL");
    if (d->width <= 0 || d->height <= 0 || d->width > 65536 || d->height > 65536)
        return fail(VAFR_E_ARG, "display size %dx%d out of range [1, 65536]", d->width, d->height);
    if (!(d->fov_x_deg > 0.0 && d->fov_x_deg < 180.0) || !(d->fov_y_deg > 0.0 && d->fov_y_deg < 180.0))
        return fail(VAFR_E_ARG, "field of view must lie in (0, 180) degrees");
    return VAFR_OK;
}

// Interleave the bits of two 16-bit integers (Morton / Z order).
static uint32_t morton2(uint32_t x, uint32_t y) {
    auto spread = [](uint32_t v) {
        v &= 0xffff;
        v = (v | (v << 8)) & 0x00ff00ff;
        v = (v | (v << 4)) & 0x0f0f0f0f;
        v = (v | (v << 2)) & 0x33333333;
        v = (v | (v << 1)) & 0x55555555;
        return v;
    };
    return spread(x) | (spread(y) << 1);
}

// Trace order: texels sorted by the Morton code of their screen offset from
// the gaze point, so that the 64 rays of a wave leave through a compact patch
// of the screen (column-major order would spread them along a long arc).
static void build_trace_order(vafr_layout_s* L) {
    const int64_t n = L->n_texels;
    float R = 0.0f;
    for (int64_t k = 0; k < 2 * n; ++k) R = std::max(R, std::fabs(L->dxy[k]));
    const double scale = R > 0.0f ? 65535.0 / (2.0 * R) : 0.0;
    std::vector<uint64_t> key(n);
    for (int64_t k = 0; k < n; ++k) {
        const uint32_t qx = (uint32_t)std::min(65535.0, (L->dxy[2 * k] + R) * scale);
        const uint32_t qy = (uint32_t)std::min(65535.0, (L->dxy[2 * k + 1] + R) * scale);
        key[k] = ((uint64_t)morton2(qx, qy) << 32) | (uint64_t)k;
    }
    std::sort(key.begin(), key.end());
    L->ord.resize(n);
    for (int64_t k = 0; k < n; ++k) L->ord[k] = (int32_t)(key[k] & 0xffffffffu);
}

int layout_resident(vafr_layout L, bool* resident) {
    int dev = -1;
    VAFR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(L->mu);
    *resident = false;
    for (auto& d : L->dev)
        if (d.device == dev) *resident = true;
    return VAFR_OK;
}

int layout_device(vafr_layout L, const LayoutDev** out) {
    int dev = -1;
    VAFR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(L->mu);
    for (auto& d : L->dev)
        if (d.device == dev) { *out = &d; return VAFR_OK; }
    LayoutDev d;
    d.device = dev;
    if (L->kind == VAFR_LAYOUT_VAFR) {
        std::vector<int2> col(L->n_cols);
        for (int i = 0; i < L->n_cols; ++i) col[i] = make_int2(L->n_rows[i], (int)L->col_off[i]);
        VAFR_HIP(hipMalloc(&d.col, sizeof(int2) * col.size()));
        VAFR_HIP(hipMemcpy(d.col, col.data(), sizeof(int2) * col.size(), hipMemcpyHostToDevice));
        std::vector<float2> dxy_ord(L->n_texels);
        for (int64_t k = 0; k < L->n_texels; ++k)
            dxy_ord[k] = make_float2(L->dxy[2 * (int64_t)L->ord[k]], L->dxy[2 * (int64_t)L->ord[k] + 1]);
        VAFR_HIP(hipMalloc(&d.dxy, sizeof(float2) * dxy_ord.size()));
        VAFR_HIP(hipMemcpy(d.dxy, dxy_ord.data(), sizeof(float2) * dxy_ord.size(), hipMemcpyHostToDevice));
        VAFR_HIP(hipMalloc(&d.dxy_tex, sizeof(float) * L->dxy.size()));
        VAFR_HIP(hipMemcpy(d.dxy_tex, L->dxy.data(), sizeof(float) * L->dxy.size(), hipMemcpyHostToDevice));
        VAFR_HIP(hipMalloc(&d.ord, sizeof(int32_t) * L->ord.size()));
        VAFR_HIP(hipMemcpy(d.ord, L->ord.data(), sizeof(int32_t) * L->ord.size(), hipMemcpyHostToDevice));
        std::vector<int32_t> blk((L->n_texels + kTexelBlock - 1) / kTexelBlock);
        for (int32_t c = 0, b = 0; b < (int32_t)blk.size(); ++b) {
            const int64_t k = (int64_t)b * kTexelBlock;
            while (c + 1 < L->n_cols && L->col_off[c + 1] <= k) ++c;
            blk[b] = c;
        }
        VAFR_HIP(hipMalloc(&d.blk_col, sizeof(int32_t) * std::max<size_t>(1, blk.size())));
        VAFR_HIP(hipMemcpy(d.blk_col, blk.data(), sizeof(int32_t) * blk.size(), hipMemcpyHostToDevice));
        VAFR_HIP(hipMalloc(&d.u_of_rho, sizeof(float) * L->u_of_rho.size()));
        VAFR_HIP(hipMemcpy(d.u_of_rho, L->u_of_rho.data(), sizeof(float) * L->u_of_rho.size(), hipMemcpyHostToDevice));
    } else {
        std::vector<double2> cs(L->max_rows);
        for (int j = 0; j < L->max_rows; ++j) cs[j] = make_double2(L->lm_cos[j], L->lm_sin[j]);
        if (!L->lm_z.empty()) {
            VAFR_HIP(hipMalloc(&d.lm_z, sizeof(double) * L->lm_z.size()));
            VAFR_HIP(hipMemcpy(d.lm_z, L->lm_z.data(), sizeof(double) * L->lm_z.size(), hipMemcpyHostToDevice));
        }
        VAFR_HIP(hipMalloc(&d.lm_cs, sizeof(double2) * cs.size()));
        VAFR_HIP(hipMemcpy(d.lm_cs, cs.data(), sizeof(double2) * cs.size(), hipMemcpyHostToDevice));
    }
    L->dev.push_back(d);
    *out = &L->dev.back();
    return VAFR_OK;
}

}  // namespace vafr

using namespace vafr;

extern "C" int vafr_lp_layout(const vafr_display* display, const vafr_acuity* acuity, vafr_layout* out) {
    if (!out) return fail(VAFR_E_ARG, "out is NULL");
    *out = nullptr;
    if (int rc = check_display(display)) return rc;
    static const double kEcc[5] = {0.0, 10.0, 20.0, 30.0, 60.0};
    static const double kCpd[5] = {40.0, 10.0, 6.0, 5.0, 4.0};
    vafr_acuity def{5, kEcc, kCpd, 60.0};
    const vafr_acuity* a = acuity ? acuity : &def;
    if (!(a->e_max_deg > 0.0 && a->e_max_deg < 90.0)) return fail(VAFR_E_ARG, "e_max must lie in (0, 90)");
    Segments seg;
    if (int rc = build_segments(a->n_pivots, a->ecc_deg, a->cpd, &seg)) return rc;
    // MAR must stay positive up to e_max (and a little beyond for corners).
    for (int k = 0; k < seg.n; ++k) {
        double hi = (k + 1 < seg.n) ? seg.e[k + 1] : std::max(seg.e[k + 1], a->e_max_deg) + 30.0;
        if (!(seg.m[k] * seg.e[k] + seg.b[k] > 0.0) || !(seg.m[k] * hi + seg.b[k] > 0.0))
            return fail(VAFR_E_ARG, "acuity model gives a non-positive MAR on segment %d", k);
    }
    if (acuity && acuity->n_aniso != 0) {
        if (acuity->n_aniso < 0 || acuity->n_aniso > kMaxSeg + 1)
            return fail(VAFR_E_ARG, "n_aniso must be in [0, %d]", kMaxSeg + 1);
        if (!acuity->aniso_ecc_deg || !acuity->aniso_delta) return fail(VAFR_E_ARG, "anisotropy arrays are NULL");
        for (int k = 0; k < acuity->n_aniso; ++k) {
            const double e = acuity->aniso_ecc_deg[k], d = acuity->aniso_delta[k];
            if (!std::isfinite(e) || !(d > 0.0 && d <= 16.0))
                return fail(VAFR_E_ARG, "anisotropy point %d: eccentricity must be finite, delta in (0, 16]", k);
            if (k && !(e > acuity->aniso_ecc_deg[k - 1]))
                return fail(VAFR_E_ARG, "anisotropy eccentricities must increase strictly");
        }
    }
    vafr_layout L = new (std::nothrow) vafr_layout_s;
    if (!L) return fail(VAFR_E_OOM, "layout allocation failed");
    L->kind = VAFR_LAYOUT_VAFR;
    if (acuity && acuity->n_aniso > 0) {
        L->aniso_e.assign(acuity->aniso_ecc_deg, acuity->aniso_ecc_deg + acuity->n_aniso);
        L->aniso_d.assign(acuity->aniso_delta, acuity->aniso_delta + acuity->n_aniso);
    }
    L->disp = *display;
    film_pitch(*display, &L->px, &L->py);
    L->seg = seg;
    L->e_max = a->e_max_deg;
    // Columns sampled at their centres u = i + 1/2; rows = ceil(l(e_i)).
    const double umax = seg_u(seg, a->e_max_deg);
    L->n_cols = (int32_t)std::ceil(umax);
    try {
        L->n_rows.resize(L->n_cols);
        L->col_off.resize(L->n_cols + 1);
        int64_t off = 0;
        std::vector<double> col_e(L->n_cols);
        for (int32_t i = 0; i < L->n_cols; ++i) {
            col_e[i] = seg_e_of_u(seg, i + 0.5);
            double h = seg_l(seg, col_e[i]);
            if (!L->aniso_e.empty()) h = aniso_delta(*L, col_e[i]) * h;
            const int32_t n = (int32_t)std::ceil(h);
            L->n_rows[i] = n < 1 ? 1 : n;
            L->col_off[i] = off;
            off += L->n_rows[i];
            if (L->n_rows[i] > L->max_rows) L->max_rows = L->n_rows[i];
        }
        L->col_off[L->n_cols] = off;
        L->n_texels = off;
        if (off >= (int64_t)1 << 31) {
            delete L;
            return fail(VAFR_E_UNSUPPORTED, "layout with %lld texels exceeds 2^31", (long long)off);
        }
        // Film offset of each texel's screen point from the gaze point:
        // radius tan(e_i) (Eq. (3) at unit focal length) along the row angle.
        L->dxy.resize(2 * (size_t)off);
        for (int32_t i = 0; i < L->n_cols; ++i) {
            const double rho = std::tan(col_e[i] * kDeg);
            const int32_t n = L->n_rows[i];
            float* d = L->dxy.data() + 2 * L->col_off[i];
            for (int32_t j = 0; j < n; ++j) {
                const double th = (360.0 * (j + 0.5) / n) * kDeg;
                d[2 * j] = (float)(rho * std::cos(th));
                d[2 * j + 1] = (float)(rho * std::sin(th));
            }
        }
        build_trace_order(L);
        // Radial table for the inverse map: u as a function of the film
        // radius rho = tan(e) (Eqs. (3), (5)), clamped to the first and last
        // column centres; beyond rho_max every pixel reads the last column.
        const double u_hi = L->n_cols - 0.5;
        L->rho_max = std::tan(seg_e_of_u(seg, u_hi) * kDeg);
        std::vector<double> u(kURhoN + 1);
        for (int k = 0; k <= kURhoN; ++k) {
            const double rho = L->rho_max * k / kURhoN;
            const double e = std::atan(rho) / kDeg;
            u[k] = std::min(std::max(seg_u(seg, e), 0.5), u_hi);
        }
        L->u_of_rho.resize(2 * (kURhoN + 1));
        for (int k = 0; k <= kURhoN; ++k) {
            L->u_of_rho[2 * k] = (float)u[k];
            L->u_of_rho[2 * k + 1] = k < kURhoN ? (float)(u[k + 1] - u[k]) : 0.0f;
        }
        // Bound on |table - u(rho)| in columns for searches that must not
        // miss a column: the interpolation error (sampled inside every
        // interval), the table's FP32 rounding, and a film-radius error of
        // 4e-7 times the steepest slope.
        double err = 0.0, slope = 0.0;
        for (int k = 0; k < kURhoN; ++k) {
            const double du = (double)L->u_of_rho[2 * k + 1];
            slope = std::max(slope, std::fabs(u[k + 1] - u[k]) * kURhoN / L->rho_max);
            for (int q = 1; q < 5; ++q) {
                const double f = 0.2 * q;
                const double rho = L->rho_max * (k + f) / kURhoN;
                const double ex = std::min(std::max(seg_u(seg, std::atan(rho) / kDeg), 0.5), u_hi);
                err = std::max(err, std::fabs((double)L->u_of_rho[2 * k] + f * du - ex));
            }
        }
        L->u_margin = 2.0 * err + 4e-7 * slope + 1e-3;
    } catch (const std::bad_alloc&) {
        delete L;
        return fail(VAFR_E_OOM, "layout tables allocation failed");
    }
    *out = L;
    return VAFR_OK;
}

// Dense log-polar buffer shared by LMFR and LaFR: round(W/delta) x
// round(H/delta) texels (Sec. 5.2: delta^2 display pixels per texel), row j
// at polar angle theta = 360 (j + 1/2)/h.
static int dense_layout(const vafr_display* display, double delta, int kind, vafr_layout* out) {
    vafr_layout L = new (std::nothrow) vafr_layout_s;
    if (!L) return fail(VAFR_E_OOM, "layout allocation failed");
    L->kind = kind;
    L->disp = *display;
    film_pitch(*display, &L->px, &L->py);
    L->delta = delta;
    const int32_t w = (int32_t)std::lround(display->width / delta);
    const int32_t h = (int32_t)std::lround(display->height / delta);
    L->n_cols = w < 1 ? 1 : w;
    L->max_rows = h < 1 ? 1 : h;
    L->n_texels = (int64_t)L->n_cols * L->max_rows;
    try {
        L->n_rows.assign(L->n_cols, L->max_rows);
        L->col_off.resize(L->n_cols + 1);
        for (int32_t i = 0; i <= L->n_cols; ++i) L->col_off[i] = (int64_t)i * L->max_rows;
        L->lm_cos.resize(L->max_rows);
        L->lm_sin.resize(L->max_rows);
        for (int32_t j = 0; j < L->max_rows; ++j) {
            const double th = 360.0 * (j + 0.5) / L->max_rows;
            L->lm_cos[j] = std::cos(th * kDeg);
            L->lm_sin[j] = std::sin(th * kDeg);
        }
    } catch (const std::bad_alloc&) {
        delete L;
        return fail(VAFR_E_OOM, "layout tables allocation failed");
    }
    *out = L;
    return VAFR_OK;
}

extern "C" int lmfr_lp_layout(const vafr_display* display, double delta, double alpha, vafr_layout* out) {
    if (!out) return fail(VAFR_E_ARG, "out is NULL");
    *out = nullptr;
    if (int rc = check_display(display)) return rc;
    if (!(delta >= 1.0 && delta < 1e6)) return fail(VAFR_E_ARG, "delta must be >= 1");
    if (!(alpha > 0.0 && alpha < 64.0)) return fail(VAFR_E_ARG, "alpha must be in (0, 64)");
    vafr_layout L;
    if (int rc = dense_layout(display, delta, VAFR_LAYOUT_LMFR, &L)) return rc;
    L->alpha = alpha;
    try {
        // Inverse of Eq. (1) with K(z) = z^alpha: column i sits at
        // z = ((i + 1/2)/w)^(1/alpha).
        L->lm_z.resize(L->n_cols);
        for (int32_t i = 0; i < L->n_cols; ++i) L->lm_z[i] = std::pow((i + 0.5) / L->n_cols, 1.0 / alpha);
    } catch (const std::bad_alloc&) {
        delete L;
        return fail(VAFR_E_OOM, "layout tables allocation failed");
    }
    *out = L;
    return VAFR_OK;
}

extern "C" int lafr_lp_layout(const vafr_display* display, double delta, double a, double alpha, double beta,
                              vafr_layout* out) {
    if (!out) return fail(VAFR_E_ARG, "out is NULL");
    *out = nullptr;
    if (int rc = check_display(display)) return rc;
    if (!(delta >= 1.0 && delta < 1e6)) return fail(VAFR_E_ARG, "delta must be >= 1");
    if (!(a > 0.0 && a < 1.0)) return fail(VAFR_E_ARG, "a must be in (0, 1)");
    if (!(alpha > 0.0 && alpha <= 1.0)) return fail(VAFR_E_ARG, "alpha must be in (0, 1]");
    if (!(beta > 0.0 && beta <= 16.0)) return fail(VAFR_E_ARG, "beta must be in (0, 16]");
    vafr_layout L;
    if (int rc = dense_layout(display, delta, VAFR_LAYOUT_LAFR, &L)) return rc;
    // The column -> z map of Eq. (15) moves with the gaze (through ln L and
    // Z_ef), so it is evaluated per ray from per-view constants.
    L->alpha = alpha;
    L->lf_a = a;
    L->lf_beta = beta;
    *out = L;
    return VAFR_OK;
}

extern "C" int vafr_layout_dims(vafr_layout L, vafr_dims* out) {
    if (!L || !out) return fail(VAFR_E_ARG, "NULL argument");
    out->kind = L->kind;
    out->n_cols = L->n_cols;
    out->max_rows = L->max_rows;
    out->width = L->disp.width;
    out->height = L->disp.height;
    out->n_texels = L->n_texels;
    return VAFR_OK;
}

extern "C" int vafr_layout_tables(vafr_layout L, const int32_t** n_rows, const int64_t** col_off,
                                  const float** texel_dxy) {
    if (!L) return fail(VAFR_E_ARG, "layout is NULL");
    if (n_rows) *n_rows = L->n_rows.data();
    if (col_off) *col_off = L->col_off.data();
    if (texel_dxy) *texel_dxy = L->kind == VAFR_LAYOUT_VAFR ? L->dxy.data() : nullptr;
    return VAFR_OK;
}

extern "C" void vafr_layout_destroy(vafr_layout L) {
    if (!L) return;
    int cur = -1;
    bool have = hipGetDevice(&cur) == hipSuccess;
    for (auto& d : L->dev) {
        if (hipSetDevice(d.device) != hipSuccess) continue;
        (void)hipFree(d.col);
        (void)hipFree(d.dxy);
        (void)hipFree(d.dxy_tex);
        (void)hipFree(d.ord);
        (void)hipFree(d.blk_col);
        (void)hipFree(d.u_of_rho);
        (void)hipFree(d.lm_z);
        (void)hipFree(d.lm_cs);
    }
    if (have) (void)hipSetDevice(cur);
    delete L;
}

extern "C" int vafr_acuity_capped(const vafr_acuity* in, double cap_cpd, double* ecc_out, double* cpd_out,
                                  int32_t max_out, int32_t* n_out) {
    if (!ecc_out || !cpd_out || !n_out) return fail(VAFR_E_ARG, "NULL output");
    *n_out = 0;
    static const double kEcc[5] = {0.0, 10.0, 20.0, 30.0, 60.0};
    static const double kCpd[5] = {40.0, 10.0, 6.0, 5.0, 4.0};
    const int n = in ? in->n_pivots : 5;
    const double* ecc = in ? in->ecc_deg : kEcc;
    const double* cpd = in ? in->cpd : kCpd;
    Segments check;
    if (int rc = build_segments(n, ecc, cpd, &check)) return rc;
    if (!(cap_cpd > 0.0) || !std::isfinite(cap_cpd)) return fail(VAFR_E_ARG, "cap_cpd must be finite and > 0");
    int32_t m = 0;
    auto push = [&](double e, double f) {
        if (m >= max_out) return false;
        ecc_out[m] = e;
        cpd_out[m] = f;
        ++m;
        return true;
    };
    // f_cap = min(f, cap) <=> MAR_cap = max(MAR, 1/cap); MAR is linear per
    // segment, so the only new corner is where it crosses 1/cap.
    const double mar_cap = 1.0 / cap_cpd;
    bool ok = push(ecc[0], std::min(cpd[0], cap_cpd));
    for (int k = 0; ok && k + 1 < n; ++k) {
        const double m0 = 1.0 / cpd[k], m1 = 1.0 / cpd[k + 1];
        if ((m0 - mar_cap) * (m1 - mar_cap) < 0.0)
            ok = push(ecc[k] + (mar_cap - m0) / (m1 - m0) * (ecc[k + 1] - ecc[k]), cap_cpd);
        if (ok) ok = push(ecc[k + 1], std::min(cpd[k + 1], cap_cpd));
    }
    if (!ok) return fail(VAFR_E_ARG, "max_out = %d is too small for the capped curve", max_out);
    *n_out = m;
    return VAFR_OK;
}
