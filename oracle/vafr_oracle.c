/*
 * vafr_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU reference for the VaFR hot path: the acuity-derived
 * log-polar (LP) layout, one primary ray per LP texel, closest hit against a
 * triangle soup, Lambert shading with one shadow ray, and the inverse map of
 * the LP buffer onto display pixels.  It also covers the LMFR and LaFR
 * log-polar comparison mappings and the full-resolution ray cast.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The product path never calls it, and it shares no
 * code, header or table with the product path.
 *
 * Citations name sections and equations of "Visual Acuity Consistent Foveated
 * Rendering towards Retinal Resolution" (Zhang, Gai, Li; arXiv 2503.23410).
 * Where the paper is silent the reading taken is stated at the point of use.
 *
 * Precision: every mapping quantity is FP64 (libm).  The ray/triangle test is
 * the FP32 watertight test of Woop, Benthin and Wald (JCGT 2013), written out
 * with every rounding stated, because that test *is* the method being checked:
 * given the same FP32 ray, it decides hits exactly.  Build with
 * -ffp-contract=off so that no multiply-add is fused unless fmaf() says so.
 *
 * Parity pins: each function below is pinned by a test in tests/ against a
 * value the paper prints, a closed form, an invariant or brute force; the
 * path-tracing shading mode is the one part whose colour values are pinned
 * only by closed-form special cases (see or_shade_path_rays).  The value of
 * the LaFR constant Fa (or_lafr_consts) rests on a reading of a garbled
 * formula and is parity unpinned; the rest of the LaFR map is pinned
 * through the shading rates the paper prints for it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAX_SEG 16
#define OR_DEG (M_PI / 180.0)

/* ------------------------------------------------------------------------ */
/* Threads                                                                    */
/* ------------------------------------------------------------------------ */

void or_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int or_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Acuity model: Sec. 3.2.1 Eq. (2), segmented per Sec. 3.3 Eq. (12)         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n_seg;
    double e_piv[OR_MAX_SEG + 1]; /* pivot eccentricities, degrees           */
    double m[OR_MAX_SEG];         /* MAR slope on segment k (deg/cycle/deg)  */
    double b[OR_MAX_SEG];         /* MAR intercept: omega_k(e) = m e + b     */
    double c[OR_MAX_SEG];         /* additive constant of u on segment k     */
    double u_piv[OR_MAX_SEG + 1]; /* u at each pivot                         */
    /* Anisotropy, Eq. (19): tangential over radial shading rate Delta(e),
     * linear between (aniso_e[k], aniso_d[k]), constant outside; n_aniso = 0
     * means Delta = 1. */
    int n_aniso;
    double aniso_e[OR_MAX_SEG + 1];
    double aniso_d[OR_MAX_SEG + 1];
} or_acuity;

int or_acuity_size(void) { return (int)sizeof(or_acuity); }

/* MAR on segment k, Eq. (2): omega = m e + omega_0 with the segment's own
 * slope and intercept (Eq. (12)). */
static double seg_omega(const or_acuity* a, int k, double e) { return a->m[k] * e + a->b[k]; }

/* Eq. (5) on segment k (Eq. (12)), before the constant c_k is added. */
static double seg_u_raw(const or_acuity* a, int k, double e) {
    if (a->m[k] == 0.0) return 2.0 * e / a->b[k];   /* limit m -> 0 of Eq. (5) */
    return 2.0 * log(seg_omega(a, k, e)) / a->m[k];
}

/*
 * Pivots -> segments.  Reading of Sec. 3.3: MAR (the reciprocal of the acuity
 * f) is linear between consecutive pivots (e_k, f_k), i.e. Eq. (2) holds on
 * each segment with omega(e_k) = 1/f_k and omega(e_{k+1}) = 1/f_{k+1}.  The
 * constants c_k follow from u(0) = 0 and continuity of u at the pivots (the
 * paper leaves c_0 and the c_k unspecified).  Returns 0 on success.
 */
int or_acuity_init(or_acuity* a, int n_piv, const double* ecc, const double* cpd) {
    if (n_piv < 2 || n_piv > OR_MAX_SEG + 1) return -1;
    if (ecc[0] != 0.0) return -1;
    for (int k = 0; k < n_piv; ++k) {
        if (!(cpd[k] > 0.0)) return -1;
        if (k > 0 && !(ecc[k] > ecc[k - 1])) return -1;
    }
    memset(a, 0, sizeof(*a));
    a->n_seg = n_piv - 1;
    for (int k = 0; k < n_piv; ++k) a->e_piv[k] = ecc[k];
    for (int k = 0; k < a->n_seg; ++k) {
        double w0 = 1.0 / cpd[k], w1 = 1.0 / cpd[k + 1];
        a->m[k] = (w1 - w0) / (ecc[k + 1] - ecc[k]);
        a->b[k] = w0 - a->m[k] * ecc[k];
    }
    a->u_piv[0] = 0.0;
    for (int k = 0; k < a->n_seg; ++k) {
        a->c[k] = a->u_piv[k] - seg_u_raw(a, k, a->e_piv[k]);
        a->u_piv[k + 1] = seg_u_raw(a, k, a->e_piv[k + 1]) + a->c[k];
    }
    return 0;
}

/* Eq. (19) multiplies the tangential coordinate v by Delta(e).  The paper
 * gives Delta no functional form; it is taken as a piecewise-linear table. */
int or_acuity_set_aniso(or_acuity* a, int n, const double* ecc, const double* delta) {
    if (n < 0 || n > OR_MAX_SEG + 1) return -1;
    for (int k = 0; k < n; ++k) {
        if (!(delta[k] > 0.0)) return -1;
        if (k > 0 && !(ecc[k] > ecc[k - 1])) return -1;
        a->aniso_e[k] = ecc[k];
        a->aniso_d[k] = delta[k];
    }
    a->n_aniso = n;
    return 0;
}

double or_delta(const or_acuity* a, double e) {
    if (a->n_aniso == 0) return 1.0;
    if (e <= a->aniso_e[0]) return a->aniso_d[0];
    for (int k = 0; k + 1 < a->n_aniso; ++k) {
        if (e < a->aniso_e[k + 1]) {
            double t = (e - a->aniso_e[k]) / (a->aniso_e[k + 1] - a->aniso_e[k]);
            return a->aniso_d[k] + t * (a->aniso_d[k + 1] - a->aniso_d[k]);
        }
    }
    return a->aniso_d[a->n_aniso - 1];
}

/* Device-adapted curve (Sec. 3.3): the acuity f(e) is held at the display's
 * limit, f_cap(e) = min(f(e), cap).  On each segment the MAR 1/f is linear,
 * so 1/f_cap = max(MAR, 1/cap) is linear too except where MAR crosses 1/cap;
 * that crossing becomes a new pivot.  Returns the number of pivots written
 * (at most max_out) or -1. */
int or_acuity_capped(int n, const double* ecc, const double* cpd, double cap, double* ecc_out, double* cpd_out,
                     int max_out) {
    if (n < 2 || !(cap > 0.0)) return -1;
    int m = 0;
#define OR_PUSH(E, F) do { if (m >= max_out) return -1; ecc_out[m] = (E); cpd_out[m] = (F); ++m; } while (0)
    OR_PUSH(ecc[0], cpd[0] < cap ? cpd[0] : cap);
    for (int k = 0; k + 1 < n; ++k) {
        double w0 = 1.0 / cpd[k], w1 = 1.0 / cpd[k + 1], wc = 1.0 / cap;
        if ((w0 - wc) * (w1 - wc) < 0.0) {
            double e = ecc[k] + (wc - w0) / (w1 - w0) * (ecc[k + 1] - ecc[k]);
            OR_PUSH(e, cap);
        }
        OR_PUSH(ecc[k + 1], cpd[k + 1] < cap ? cpd[k + 1] : cap);
    }
#undef OR_PUSH
    return m;
}

/* Segment holding eccentricity e; the last segment extends past the last
 * pivot (needed for the last partial column and off-axis corners). */
static int seg_of_e(const or_acuity* a, double e) {
    int k = 0;
    while (k < a->n_seg - 1 && e >= a->e_piv[k + 1]) ++k;
    return k;
}

static int seg_of_u(const or_acuity* a, double u) {
    int k = 0;
    while (k < a->n_seg - 1 && u >= a->u_piv[k + 1]) ++k;
    return k;
}

/* Eq. (2): minimum angle of resolution at eccentricity e (degrees). */
double or_omega(const or_acuity* a, double e) { return seg_omega(a, seg_of_e(a, e), e); }

/* Eq. (5) / Eq. (12): LP abscissa of eccentricity e (degrees). */
double or_u(const or_acuity* a, double e) {
    int k = seg_of_e(a, e);
    return seg_u_raw(a, k, e) + a->c[k];
}

/* Eq. (10), segmented as Sec. 3.3 states: eccentricity of LP abscissa u. */
double or_e_of_u(const or_acuity* a, double u) {
    int k = seg_of_u(a, u);
    if (a->m[k] == 0.0) return (u - a->c[k]) * a->b[k] / 2.0;
    return (exp((u - a->c[k]) * a->m[k] / 2.0) - a->b[k]) / a->m[k];
}

/* Eq. (9): shading height l(e) = 360 sin(2e) / omega(e), angles in degrees. */
double or_l(const or_acuity* a, double e) { return 360.0 * sin(2.0 * e * OR_DEG) / or_omega(a, e); }

/* Eq. (8): LP ordinate of a point at eccentricity e and polar angle theta. */
double or_v(const or_acuity* a, double e, double theta) {
    return theta * sin(2.0 * e * OR_DEG) / or_omega(a, e);
}

void or_u_many(const or_acuity* a, const double* e, int64_t n, double* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = or_u(a, e[i]);
}
void or_e_many(const or_acuity* a, const double* u, int64_t n, double* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = or_e_of_u(a, u[i]);
}
void or_l_many(const or_acuity* a, const double* e, int64_t n, double* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = or_l(a, e[i]);
}
void or_omega_many(const or_acuity* a, const double* e, int64_t n, double* out) {
    for (int64_t i = 0; i < n; ++i) out[i] = or_omega(a, e[i]);
}

/* ------------------------------------------------------------------------ */
/* Constant-size LP buffer: Sec. 3.2.2                                        */
/* ------------------------------------------------------------------------ */

/*
 * Discretisation (the paper gives the continuous sizes u(e_max) and l(e) but
 * not the sampling): there are ceil(u(e_max)) columns; column i is sampled at
 * its centre u = i + 1/2, i.e. at eccentricity e_i = e(i + 1/2) (Eq. (10));
 * it holds n_i = ceil(l(e_i)) texels (Eq. (9)), rounded up so the tangential
 * rate never drops below the acuity model; row j sits at polar angle
 * theta_ij = 360 (j + 1/2) / n_i degrees so the rows tile the full circle.
 */
/* Rows of a column at eccentricity e: the shading height l(e) of Eq. (9),
 * times Delta(e) when the tangential rate is anisotropic (Eq. (19)),
 * rounded up so that the tangential rate is never below the model. */
static int32_t or_rows(const or_acuity* a, double e) {
    double h = or_l(a, e);
    if (a->n_aniso > 0) h = or_delta(a, e) * h;
    int32_t n = (int32_t)ceil(h);
    return n < 1 ? 1 : n;
}

int or_vafr_layout_dims(const or_acuity* a, double e_max, int32_t* n_cols, int64_t* n_texels) {
    double umax = or_u(a, e_max);
    int32_t nc = (int32_t)ceil(umax);
    int64_t tot = 0;
    for (int32_t i = 0; i < nc; ++i) {
        double e = or_e_of_u(a, i + 0.5);
        tot += or_rows(a, e);
    }
    *n_cols = nc;
    *n_texels = tot;
    return 0;
}

/*
 * Tables of the layout.  dxy holds, per texel in column-major order
 * (all rows of column 0, then column 1, ...), the film-plane offset of the
 * texel's screen point from the gaze point, in units of the focal length:
 * rho = tan e_i (Eq. (3) with the pixel pitch factored out) along the
 * direction theta_ij (Eq. (11)).  FP64 throughout, rounded to FP32 once.
 */
int or_vafr_layout_fill(const or_acuity* a, double e_max, int32_t n_cols, int32_t* n_rows,
                        int64_t* col_off, float* dxy, double* col_e) {
    (void)e_max;
    int64_t off = 0;
    for (int32_t i = 0; i < n_cols; ++i) {
        double e = or_e_of_u(a, i + 0.5);
        int32_t n = or_rows(a, e);
        n_rows[i] = n;
        col_off[i] = off;
        if (col_e) col_e[i] = e;
        double rho = tan(e * OR_DEG);
        if (dxy) {
            for (int32_t j = 0; j < n; ++j) {
                double th = 360.0 * (j + 0.5) / n;
                dxy[2 * (off + j) + 0] = (float)(rho * cos(th * OR_DEG));
                dxy[2 * (off + j) + 1] = (float)(rho * sin(th * OR_DEG));
            }
        }
        off += n;
    }
    col_off[n_cols] = off;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Display <-> film plane (Sec. 3.2.1, Eq. (3))                              */
/* ------------------------------------------------------------------------ */

/*
 * Eq. (3) converts a pixel distance r to eccentricity with the constant c_r
 * (film height / focal length / display height).  The display may have
 * non-square pixels (a 16:9 panel with a square field of view), so the
 * conversion is kept per axis: the film plane is at unit focal length and a
 * pixel spans px = 2 tan(fov_x/2) / W horizontally and py = 2 tan(fov_y/2)/H
 * vertically; for square pixels c_r = py.  Screen x grows right, y grows down;
 * the continuous pixel point (x, y) maps to ((x - W/2) px, (y - H/2) py).
 */
void or_film_pitch(int32_t W, int32_t H, double fov_x_deg, double fov_y_deg, double* p) {
    p[0] = 2.0 * tan(0.5 * fov_x_deg * OR_DEG) / W;
    p[1] = 2.0 * tan(0.5 * fov_y_deg * OR_DEG) / H;
}

void or_gaze_film(int32_t W, int32_t H, const double* p, double gx, double gy, double* G) {
    G[0] = (gx - 0.5 * W) * p[0];
    G[1] = (gy - 0.5 * H) * p[1];
}

/*
 * Forward map of a continuous pixel point to LP coordinates:
 * e = atan(rho) (Eq. (3)), theta = polar angle of the offset from the gaze
 * measured from +x toward +y (screen down) in [0, 360), u = u(e) (Eq. (5)),
 * v = v(e, theta) (Eq. (8)).  Eccentricity is the angle subtended at the eye
 * by the film-plane distance from the gaze point (the paper's Eq. (3) read
 * literally), which keeps the map a translation of the gaze point.
 */
void or_vafr_forward(const or_acuity* a, int32_t W, int32_t H, const double* p, const double* G,
                     int64_t n, const double* xy, double* u, double* v, double* e_out, double* th_out) {
    for (int64_t i = 0; i < n; ++i) {
        double X = (xy[2 * i] - 0.5 * W) * p[0];
        double Y = (xy[2 * i + 1] - 0.5 * H) * p[1];
        double dx = X - G[0], dy = Y - G[1];
        double rho = sqrt(dx * dx + dy * dy);
        double e = atan(rho) / OR_DEG;
        double th = atan2(dy, dx) / OR_DEG;
        if (th < 0.0) th += 360.0;
        if (u) u[i] = or_u(a, e);
        if (v) v[i] = or_v(a, e, th);
        if (e_out) e_out[i] = e;
        if (th_out) th_out[i] = th;
    }
}

/*
 * Inverse map, Eqs. (10)-(11): e from u, theta = 360 v / l(e), then the
 * screen point at film distance tan e from the gaze along theta.
 */
void or_vafr_inverse(const or_acuity* a, int32_t W, int32_t H, const double* p, const double* G,
                     int64_t n, const double* u, const double* v, double* xy) {
    for (int64_t i = 0; i < n; ++i) {
        double e = or_e_of_u(a, u[i]);
        double th = 360.0 * v[i] / or_l(a, e);
        double rho = tan(e * OR_DEG);
        double X = G[0] + rho * cos(th * OR_DEG);
        double Y = G[1] + rho * sin(th * OR_DEG);
        xy[2 * i] = X / p[0] + 0.5 * W;
        xy[2 * i + 1] = Y / p[1] + 0.5 * H;
    }
}

/* ------------------------------------------------------------------------ */
/* Rays                                                                       */
/* ------------------------------------------------------------------------ */

/*
 * A primary ray leaves the eye (pinhole) through the continuous film point
 * P = (Px, Py) (Sec. 6.1: a ray per LP texel from its screen position).
 * Camera basis: right R, up U, forward F (unit focal length), film y down.
 * The direction  D = Px R - Py U + F  is formed in FP64 from the FP32 basis,
 * operation by operation ((Px*R - Py*U) + F, no fused multiply-add), and
 * rounded to FP32 once; it is not normalised (the hit test does not need it).
 * cam = {eye[3], right[3], up[3], forward[3]}.
 */
static void make_ray(const float* cam, double Px, double Py, float* o, float* d) {
    for (int k = 0; k < 3; ++k) {
        double a = Px * (double)cam[3 + k];
        double b = Py * (double)cam[6 + k];
        double s = a - b;
        double t = s + (double)cam[9 + k];
        o[k] = cam[k];
        d[k] = (float)t;
    }
}

/* VaFR: texel k's ray passes through P = G + dxy[k] (Sec. 6.1). */
void or_vafr_rays(const float* dxy, const int64_t* idx, int64_t n, const double* G, const float* cam,
                  float* org, float* dir) {
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = idx[i];
        double Px = G[0] + (double)dxy[2 * k];
        double Py = G[1] + (double)dxy[2 * k + 1];
        make_ray(cam, Px, Py, org + 3 * i, dir + 3 * i);
    }
}

/* Full resolution: one ray through each display pixel centre. */
void or_full_rays(int32_t W, int32_t H, const double* p, const int64_t* pix, int64_t n, const float* cam,
                  float* org, float* dir) {
    for (int64_t i = 0; i < n; ++i) {
        int64_t x = pix[i] % W, y = pix[i] / W;
        double Px = ((double)x + 0.5 - 0.5 * W) * p[0];
        double Py = ((double)y + 0.5 - 0.5 * H) * p[1];
        make_ray(cam, Px, Py, org + 3 * i, dir + 3 * i);
    }
}

/* ------------------------------------------------------------------------ */
/* LMFR log-polar comparison mapping: Sec. 3.1 Eq. (1), Sec. 4.1 Eq. (14)    */
/* ------------------------------------------------------------------------ */

/* LP buffer of the comparison: (W/delta) x (H/delta), rounded to the nearest
 * integer (Sec. 2.1 and Sec. 5.2: delta^2 is the ratio of display pixels to
 * LP pixels). */
void or_lmfr_dims(int32_t W, int32_t H, double delta, int32_t* w, int32_t* h) {
    *w = (int32_t)lround(W / delta);
    *h = (int32_t)lround(H / delta);
}

/* L of Eq. (1): the log of the longest distance (pixels) from the gaze point
 * to a screen corner. */
double or_lmfr_L(int32_t W, int32_t H, double gx, double gy) {
    double best = 0.0;
    const double cx[4] = {0.0, (double)W, 0.0, (double)W};
    const double cy[4] = {0.0, 0.0, (double)H, (double)H};
    for (int c = 0; c < 4; ++c) {
        double dx = cx[c] - gx, dy = cy[c] - gy;
        double d = sqrt(dx * dx + dy * dy);
        if (d > best) best = d;
    }
    return log(best);
}

/*
 * Inverse of Eq. (1) with the LMFR kernel K(z) = z^alpha (Eq. (14), alpha =
 * 4): texel (i, j) of the w x h buffer (column-major, k = i h + j) sits at
 * z = ((i + 1/2)/w)^(1/alpha), pixel radius r = exp(L z) and polar angle
 * theta = 360 (j + 1/2)/h from the gaze; its ray goes through
 * P = G + (r cos theta px, r sin theta py).
 */
void or_lmfr_rays(int32_t W, int32_t H, const double* p, double gx, double gy, int32_t w, int32_t h,
                  double alpha, const int64_t* idx, int64_t n, const float* cam, float* org, float* dir) {
    double L = or_lmfr_L(W, H, gx, gy);
    double G[2];
    or_gaze_film(W, H, p, gx, gy, G);
    for (int64_t q = 0; q < n; ++q) {
        int64_t k = idx[q];
        int64_t i = k / h, j = k % h;
        double z = pow((i + 0.5) / w, 1.0 / alpha);
        double r = exp(L * z);
        double th = 360.0 * (j + 0.5) / h;
        double Px = G[0] + (r * cos(th * OR_DEG)) * p[0];
        double Py = G[1] + (r * sin(th * OR_DEG)) * p[1];
        make_ray(cam, Px, Py, org + 3 * q, dir + 3 * q);
    }
}

/* Forward map of Eq. (1) with K(z) = z^alpha for continuous pixel points;
 * the radius is clamped to >= 1 pixel so that z >= 0. */
void or_lmfr_forward(int32_t W, int32_t H, double gx, double gy, int32_t w, int32_t h, double alpha,
                     int64_t n, const double* xy, double* u, double* v) {
    double L = or_lmfr_L(W, H, gx, gy);
    for (int64_t q = 0; q < n; ++q) {
        double dx = xy[2 * q] - gx, dy = xy[2 * q + 1] - gy;
        double r = sqrt(dx * dx + dy * dy);
        if (r < 1.0) r = 1.0;
        double z = log(r) / L;
        double th = atan2(dy, dx) / OR_DEG;
        if (th < 0.0) th += 360.0;
        u[q] = pow(z, alpha) * w;
        v[q] = th / 360.0 * h;
    }
}

/* ------------------------------------------------------------------------ */
/* LaFR log-polar comparison mapping: Sec. 4.1 Eq. (15), Eq. (17)            */
/* ------------------------------------------------------------------------ */

/* Foveal boundary of the LaFR kernel (Sec. 4.1, Eq. (15)), degrees. */
#define OR_LAFR_FOVEAL_DEG 4.89

/*
 * Constants of Eq. (15) for one gaze, written to out[4] = {ln L, Z_ef, Fa,
 * U_ef}:
 *  - ln L as in Eq. (1) (or_lmfr_L);
 *  - z(e) = ln(tan e / c_r) / ln L with c_r the film pitch of one pixel
 *    (p[1]), so Z_ef = z(4.89 deg);
 *  - Fa = 1 - log_{Z_ef}((alpha Z_ef)^(1 - a) / (1 - a));
 *  - U_ef = (Z_ef (1 - Fa))^(1 / Fa).
 * Reading: the paper equates LaFR's a with LMFR's kernel exponent; the
 * printed Fa has a real value only for a < 1, so a is that exponent in the
 * buffer-to-screen direction (z = (u/w)^(1/4) for LMFR's z^4), i.e. 1/4.
 * Returns 0, or -1 when Z_ef or Fa lies outside (0, 1) (the kernel is then
 * undefined).
 */
int or_lafr_consts(int32_t W, int32_t H, const double* p, double gx, double gy, double a, double alpha,
                   double* out) {
    double lnL = or_lmfr_L(W, H, gx, gy);
    double r_ef = tan(OR_LAFR_FOVEAL_DEG * OR_DEG) / p[1];
    double Zef = log(r_ef) / lnL;
    double Fa = 1.0 - log(pow(alpha * Zef, 1.0 - a) / (1.0 - a)) / log(Zef);
    double Uef = pow(Zef * (1.0 - Fa), 1.0 / Fa);
    out[0] = lnL;
    out[1] = Zef;
    out[2] = Fa;
    out[3] = Uef;
    if (!(lnL > 0.0) || !(Zef > 0.0 && Zef < 1.0) || !(Fa > 0.0 && Fa < 1.0)) return -1;
    return 0;
}

/* Eq. (15): u / w at log ratio z in [0, 1], for constants c of
 * or_lafr_consts.  The first piece covers e <= 4.89 deg (z <= Z_ef), the
 * second the rest of the screen. */
static double lafr_u(const double* c, double beta, double z) {
    double Zef = c[1], Fa = c[2], Uef = c[3];
    if (z <= Zef) return pow(z * (1.0 - Fa), 1.0 / Fa);
    double Za = (1.0 / z - 1.0 / Zef) / (1.0 / Zef - 1.0);
    if (Za < -1.0) Za = -1.0;
    return pow((2.0 * acos(Za) - M_PI) / M_PI, beta / 0.7) * (1.0 - Uef) + Uef;
}

/* Inverse of Eq. (15): the log ratio z at which u / w = t (0 < t < 1).
 * First piece: z = t^Fa / (1 - Fa).  Second piece: s = ((t - U_ef) /
 * (1 - U_ef))^(0.7 / beta) is (2 acos(Za) - pi) / pi, so Za =
 * cos(pi (s + 1) / 2), and 1/z = 1/Z_ef + Za (1/Z_ef - 1). */
static double lafr_z(const double* c, double beta, double t) {
    double Zef = c[1], Fa = c[2], Uef = c[3];
    if (t <= Uef) return pow(t, Fa) / (1.0 - Fa);
    double s = pow((t - Uef) / (1.0 - Uef), 0.7 / beta);
    double Za = cos(0.5 * M_PI * (s + 1.0));
    return 1.0 / (1.0 / Zef + Za * (1.0 / Zef - 1.0));
}

void or_lafr_u(const double* c, double beta, int64_t n, const double* z, double* u) {
    for (int64_t q = 0; q < n; ++q) u[q] = lafr_u(c, beta, z[q]);
}

void or_lafr_z(const double* c, double beta, int64_t n, const double* t, double* z) {
    for (int64_t q = 0; q < n; ++q) z[q] = lafr_z(c, beta, t[q]);
}

/*
 * LaFR rays: texel (i, j) of the w x h buffer (k = i h + j) sits at
 * z = lafr_z((i + 1/2)/w), pixel radius r = exp(z ln L) and polar angle
 * theta = 360 (j + 1/2)/h from the gaze, through P = G + (r cos theta px,
 * r sin theta py).  Returns or_lafr_consts' status.
 */
int or_lafr_rays(int32_t W, int32_t H, const double* p, double gx, double gy, int32_t w, int32_t h, double a,
                 double alpha, double beta, const int64_t* idx, int64_t n, const float* cam, float* org,
                 float* dir) {
    double c[4];
    if (or_lafr_consts(W, H, p, gx, gy, a, alpha, c)) return -1;
    double G[2];
    or_gaze_film(W, H, p, gx, gy, G);
    for (int64_t q = 0; q < n; ++q) {
        int64_t k = idx[q];
        int64_t i = k / h, j = k % h;
        double z = lafr_z(c, beta, (i + 0.5) / w);
        double r = exp(c[0] * z);
        double th = 360.0 * (j + 0.5) / h;
        double Px = G[0] + (r * cos(th * OR_DEG)) * p[0];
        double Py = G[1] + (r * sin(th * OR_DEG)) * p[1];
        make_ray(cam, Px, Py, org + 3 * q, dir + 3 * q);
    }
    return 0;
}

/* Forward map of Eq. (15) for continuous pixel points (radius clamped to
 * >= 1 pixel so that z >= 0): u in columns, v in rows. */
int or_lafr_forward(int32_t W, int32_t H, const double* p, double gx, double gy, int32_t w, int32_t h, double a,
                    double alpha, double beta, int64_t n, const double* xy, double* u, double* v) {
    double c[4];
    if (or_lafr_consts(W, H, p, gx, gy, a, alpha, c)) return -1;
    for (int64_t q = 0; q < n; ++q) {
        double dx = xy[2 * q] - gx, dy = xy[2 * q + 1] - gy;
        double r = sqrt(dx * dx + dy * dy);
        if (r < 1.0) r = 1.0;
        double z = log(r) / c[0];
        double th = atan2(dy, dx) / OR_DEG;
        if (th < 0.0) th += 360.0;
        u[q] = lafr_u(c, beta, z) * w;
        v[q] = th / 360.0 * h;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2(1), 2013)       */
/* ------------------------------------------------------------------------ */

typedef struct {
    int kx, ky, kz;
    float Sx, Sy, Sz;
    int valid;
} or_shear;

/* Per-ray set-up: the axis of largest |d| becomes z (first such axis on
 * ties), x and y follow cyclically and swap when d_z < 0 to keep the winding;
 * the shear constants are correctly rounded FP32 quotients. */
static void shear_init(const float* d, or_shear* s) {
    int kz = 0;
    if (fabsf(d[1]) > fabsf(d[kz])) kz = 1;
    if (fabsf(d[2]) > fabsf(d[kz])) kz = 2;
    int kx = kz + 1 == 3 ? 0 : kz + 1;
    int ky = kx + 1 == 3 ? 0 : kx + 1;
    if (d[kz] < 0.0f) { int t = kx; kx = ky; ky = t; }
    s->kx = kx; s->ky = ky; s->kz = kz;
    s->valid = d[kz] != 0.0f;
    if (s->valid) {
        s->Sx = d[kx] / d[kz];
        s->Sy = d[ky] / d[kz];
        s->Sz = 1.0f / d[kz];
    }
}

typedef struct {
    int hit;       /* edge test passed, det != 0 and t > 0 */
    float t;       /* T / det, in units of |d|             */
    double margin; /* hits: min edge weight / sum; misses: outside weight / sum */
    int t_pos;     /* T / det > 0 (meaningful when det != 0) */
} or_tri_res;

/*
 * Arithmetic (all FP32 unless stated):
 *   A = v0 - o, B = v1 - o, C = v2 - o
 *   Ax = fma(-Sx, A_kz, A_kx), Ay = fma(-Sy, A_kz, A_ky)     (same for B, C)
 *   U = Cx By - Cy Bx, V = Ax Cy - Ay Cx, W = Bx Ay - By Ax  (no fused ops,
 *       so an edge shared by two triangles gets exactly negated values)
 *   if any of U, V, W is exactly zero: recompute all three from the FP32
 *       operands in FP64 and round each to FP32
 *   mixed signs -> miss (two-sided test); det = (U + V) + W; det == 0 -> miss
 *   T = (U Sz A_kz + V Sz B_kz) + W Sz C_kz   (each Sz * _kz rounded first)
 *   t = T / det (correctly rounded); hit iff t > 0.
 */
static void watertight(const float* o, const float* d, const or_shear* s, const float* v0,
                       const float* v1, const float* v2, or_tri_res* r) {
    (void)d; /* the ray enters only through its shear constants */
    r->hit = 0;
    r->t = INFINITY;
    r->margin = 1.0;
    r->t_pos = 0;
    if (!s->valid) return;
    const int kx = s->kx, ky = s->ky, kz = s->kz;
    float A[3], B[3], C[3];
    for (int k = 0; k < 3; ++k) {
        A[k] = v0[k] - o[k];
        B[k] = v1[k] - o[k];
        C[k] = v2[k] - o[k];
    }
    float Ax = fmaf(-s->Sx, A[kz], A[kx]);
    float Ay = fmaf(-s->Sy, A[kz], A[ky]);
    float Bx = fmaf(-s->Sx, B[kz], B[kx]);
    float By = fmaf(-s->Sy, B[kz], B[ky]);
    float Cx = fmaf(-s->Sx, C[kz], C[kx]);
    float Cy = fmaf(-s->Sy, C[kz], C[ky]);
    float p1, p2;
    p1 = Cx * By; p2 = Cy * Bx; float U = p1 - p2;
    p1 = Ax * Cy; p2 = Ay * Cx; float V = p1 - p2;
    p1 = Bx * Ay; p2 = By * Ax; float W = p1 - p2;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    int neg = (U < 0.0f) || (V < 0.0f) || (W < 0.0f);
    int pos = (U > 0.0f) || (V > 0.0f) || (W > 0.0f);
    double aU = fabs((double)U), aV = fabs((double)V), aW = fabs((double)W);
    double S = aU + aV + aW;
    float det = (U + V) + W;
    float Az = s->Sz * A[kz];
    float Bz = s->Sz * B[kz];
    float Cz = s->Sz * C[kz];
    float T = (U * Az + V * Bz) + W * Cz;
    float t = det != 0.0f ? T / det : INFINITY;
    r->t = t;
    r->t_pos = det != 0.0f && t > 0.0f;
    if (S > 0.0) {
        if (neg && pos) {
            double sn = (U < 0.0f ? aU : 0.0) + (V < 0.0f ? aV : 0.0) + (W < 0.0f ? aW : 0.0);
            double sp = S - sn;
            r->margin = (sn < sp ? sn : sp) / S;
        } else {
            double mn = aU < aV ? aU : aV;
            mn = mn < aW ? mn : aW;
            r->margin = mn / S;
        }
    }
    if (neg && pos) return;
    if (det == 0.0f) return;
    r->hit = t > 0.0f;
}

/* Test-visible form: n rays x one triangle each (used by the pins). */
void or_watertight_many(int64_t n, const float* org, const float* dir, const float* tri9, int32_t* hit,
                        float* t, double* margin) {
    for (int64_t i = 0; i < n; ++i) {
        or_shear s;
        or_tri_res r;
        shear_init(dir + 3 * i, &s);
        watertight(org + 3 * i, dir + 3 * i, &s, tri9 + 9 * i, tri9 + 9 * i + 3, tri9 + 9 * i + 6, &r);
        hit[i] = r.hit;
        t[i] = r.t;
        margin[i] = r.margin;
    }
}

/* ------------------------------------------------------------------------ */
/* Scene and the oracle's own BVH (spatial-midpoint splits, FP64 boxes)     */
/* ------------------------------------------------------------------------ */

typedef struct {
    double lo[3], hi[3];
    int64_t left, right;  /* children; -1 for a leaf */
    int64_t first, count; /* leaf triangle range in perm[] */
} or_node;

typedef struct {
    int64_t n_tris;
    float* tv;           /* 9 floats per triangle, original order and winding */
    int use_bvh;
    or_node* nodes;
    int64_t n_nodes, cap_nodes;
    int64_t* perm;
    int max_depth;
    double pad;          /* absolute box padding */
} or_scene;

static void tri_bounds(const or_scene* sc, int64_t t, double* lo, double* hi) {
    const float* v = sc->tv + 9 * t;
    for (int k = 0; k < 3; ++k) {
        double a = v[k], b = v[3 + k], c = v[6 + k];
        double mn = a < b ? a : b; mn = mn < c ? mn : c;
        double mx = a > b ? a : b; mx = mx > c ? mx : c;
        lo[k] = mn; hi[k] = mx;
    }
}

static int64_t new_node(or_scene* sc) {
    if (sc->n_nodes == sc->cap_nodes) {
        sc->cap_nodes = sc->cap_nodes ? 2 * sc->cap_nodes : 1024;
        sc->nodes = (or_node*)realloc(sc->nodes, sc->cap_nodes * sizeof(or_node));
    }
    return sc->n_nodes++;
}

/* Top-down build: split at the midpoint of the centroid bounds along their
 * widest axis; if that leaves one side empty, split the range in half.
 * Leaves hold at most 4 triangles.  Box padding makes every box test
 * conservative (the FP64 slab test's own error is far below the padding). */
static int64_t build_rec(or_scene* sc, double* cen, int64_t first, int64_t count, int depth) {
    int64_t id = new_node(sc);
    if (depth > sc->max_depth) sc->max_depth = depth;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t q = first; q < first + count; ++q) {
        double tlo[3], thi[3];
        int64_t t = sc->perm[q];
        tri_bounds(sc, t, tlo, thi);
        for (int k = 0; k < 3; ++k) {
            if (tlo[k] < lo[k]) lo[k] = tlo[k];
            if (thi[k] > hi[k]) hi[k] = thi[k];
            double c = cen[3 * t + k];
            if (c < clo[k]) clo[k] = c;
            if (c > chi[k]) chi[k] = c;
        }
    }
    or_node nd;
    for (int k = 0; k < 3; ++k) { nd.lo[k] = lo[k] - sc->pad; nd.hi[k] = hi[k] + sc->pad; }
    nd.left = nd.right = -1;
    nd.first = first;
    nd.count = count;
    if (count <= 4) { sc->nodes[id] = nd; return id; }
    int ax = 0;
    for (int k = 1; k < 3; ++k)
        if (chi[k] - clo[k] > chi[ax] - clo[ax]) ax = k;
    double mid = 0.5 * (clo[ax] + chi[ax]);
    int64_t i = first, j = first + count - 1;
    while (i <= j) {
        if (cen[3 * sc->perm[i] + ax] < mid) ++i;
        else { int64_t tmp = sc->perm[i]; sc->perm[i] = sc->perm[j]; sc->perm[j] = tmp; --j; }
    }
    int64_t nl = i - first;
    if (nl == 0 || nl == count) nl = count / 2;
    int64_t l = build_rec(sc, cen, first, nl, depth + 1);
    int64_t r = build_rec(sc, cen, first + nl, count - nl, depth + 1);
    nd.left = l; nd.right = r; nd.count = 0;
    sc->nodes[id] = nd;
    return id;
}

or_scene* or_scene_create(const float* xyz, int64_t n_verts, const int32_t* tri, int64_t n_tris, int use_bvh) {
    or_scene* sc = (or_scene*)calloc(1, sizeof(or_scene));
    sc->n_tris = n_tris;
    sc->tv = (float*)malloc((size_t)(n_tris > 0 ? n_tris : 1) * 9 * sizeof(float));
    double ext = 0.0;
    for (int64_t t = 0; t < n_tris; ++t)
        for (int c = 0; c < 3; ++c) {
            int64_t vi = tri[3 * t + c];
            if (vi < 0 || vi >= n_verts) { free(sc->tv); free(sc); return NULL; }
            for (int k = 0; k < 3; ++k) {
                float f = xyz[3 * vi + k];
                sc->tv[9 * t + 3 * c + k] = f;
                if (fabs((double)f) > ext) ext = fabs((double)f);
            }
        }
    sc->pad = 1e-5 * (1.0 + ext);
    sc->use_bvh = use_bvh && n_tris > 0;
    if (sc->use_bvh) {
        sc->perm = (int64_t*)malloc(n_tris * sizeof(int64_t));
        double* cen = (double*)malloc(3 * n_tris * sizeof(double));
        for (int64_t t = 0; t < n_tris; ++t) {
            sc->perm[t] = t;
            const float* v = sc->tv + 9 * t;
            for (int k = 0; k < 3; ++k) cen[3 * t + k] = ((double)v[k] + (double)v[3 + k] + (double)v[6 + k]) / 3.0;
        }
        build_rec(sc, cen, 0, n_tris, 0);
        free(cen);
    }
    return sc;
}

void or_scene_destroy(or_scene* sc) {
    if (!sc) return;
    free(sc->tv); free(sc->nodes); free(sc->perm); free(sc);
}

int64_t or_scene_nodes(const or_scene* sc) { return sc->n_nodes; }
int or_scene_depth(const or_scene* sc) { return sc->max_depth; }

/* FP64 slab test against the padded box over [0, tmax]. */
static int box_hit(const or_node* nd, const float* o, const float* d, double tmax) {
    double tn = 0.0, tf = tmax;
    for (int k = 0; k < 3; ++k) {
        double ok = o[k], dk = d[k];
        if (dk == 0.0) {
            if (ok < nd->lo[k] || ok > nd->hi[k]) return 0;
            continue;
        }
        double t0 = (nd->lo[k] - ok) / dk, t1 = (nd->hi[k] - ok) / dk;
        if (t0 > t1) { double tmp = t0; t0 = t1; t1 = tmp; }
        if (t0 > tn) tn = t0;
        if (t1 < tf) tf = t1;
        if (tn > tf) return 0;
    }
    return 1;
}

#define OR_TIE 1e-6

typedef struct {
    int32_t id;       /* winner, -1 on miss */
    float t;
    double margin;    /* winner's edge margin */
    float t2;         /* runner-up hit t */
    float t_near_miss;/* smallest t among near-miss candidates in front */
} or_closest;

static void visit_closest(const or_scene* sc, int64_t tri_id, const float* o, const float* d,
                          const or_shear* s, or_closest* c) {
    const float* v = sc->tv + 9 * tri_id;
    or_tri_res r;
    watertight(o, d, s, v, v + 3, v + 6, &r);
    if (r.hit) {
        int32_t id = (int32_t)tri_id;
        if (c->id < 0 || r.t < c->t || (r.t == c->t && id < c->id)) {
            if (c->id >= 0 && c->t < c->t2) c->t2 = c->t;
            c->id = id; c->t = r.t; c->margin = r.margin;
        } else if (r.t < c->t2) {
            c->t2 = r.t;
        }
    } else if (r.margin < OR_TIE && r.t_pos) {
        if (r.t < c->t_near_miss) c->t_near_miss = r.t;
    }
}

/*
 * Closest hit: the winner is the smallest (t, triangle id) over all
 * triangles hit with t > 0 (two-sided; equal t broken by the smaller id).
 * flag = 1 marks a near tie: the winner's smallest barycentric weight is
 * below 1e-6, a second hit lies within a relative 1e-6 in t, or a triangle
 * missed by less than 1e-6 (normalised barycentric) lies in front of the
 * winner (or anywhere along a missing ray).
 */
static void closest(const or_scene* sc, const float* o, const float* d, or_closest* c, uint8_t* flag) {
    or_shear s;
    shear_init(d, &s);
    c->id = -1; c->t = INFINITY; c->margin = 1.0; c->t2 = INFINITY; c->t_near_miss = INFINITY;
    if (!sc->use_bvh) {
        for (int64_t t = 0; t < sc->n_tris; ++t) visit_closest(sc, t, o, d, &s, c);
    } else {
        int64_t stack[256];
        int sp = 0;
        int64_t* big = NULL;
        int64_t* st = stack;
        int cap = 256;
        if (sc->max_depth + 2 > cap) {
            cap = sc->max_depth + 2;
            big = (int64_t*)malloc(cap * sizeof(int64_t));
            st = big;
        }
        st[sp++] = 0;
        while (sp) {
            const or_node* nd = sc->nodes + st[--sp];
            double tmax = c->id >= 0 ? (double)c->t * (1.0 + 4.0 * OR_TIE) : INFINITY;
            if (!box_hit(nd, o, d, tmax)) continue;
            if (nd->left < 0) {
                for (int64_t q = nd->first; q < nd->first + nd->count; ++q)
                    visit_closest(sc, sc->perm[q], o, d, &s, c);
            } else {
                st[sp++] = nd->right;
                st[sp++] = nd->left;
            }
        }
        free(big);
    }
    uint8_t f = 0;
    if (c->id >= 0) {
        if (c->margin < OR_TIE) f = 1;
        if (c->t2 != INFINITY && ((double)c->t2 - (double)c->t) <= OR_TIE * (double)c->t) f = 1;
        if (c->t_near_miss != INFINITY && (double)c->t_near_miss <= (double)c->t * (1.0 + OR_TIE)) f = 1;
    } else if (c->t_near_miss != INFINITY) {
        f = 1;
    }
    *flag = f;
}

/* Any hit with t > 0 (shadow ray).  Returns 1 iff some triangle passes the
 * test.  The search stops at the first hit whose edge margin is at least 1e-6;
 * otherwise every candidate is visited, so the answer is exact either way.
 * flag = 1 when no such robust hit exists but some triangle in front is hit
 * or missed within that margin. */
static int anyhit(const or_scene* sc, const float* o, const float* d, uint8_t* flag) {
    or_shear s;
    shear_init(d, &s);
    int robust = 0, near = 0, hit = 0;
    int64_t stack[256];
    int64_t* big = NULL;
    int64_t* st = stack;
    int sp = 0;
    if (sc->use_bvh && sc->max_depth + 2 > 256) {
        big = (int64_t*)malloc((sc->max_depth + 2) * sizeof(int64_t));
        st = big;
    }
    int done_linear = 0;
    if (sc->use_bvh) st[sp++] = 0;
    while (!robust) {
        int64_t first, count;
        if (!sc->use_bvh) {
            if (done_linear) break;
            first = 0; count = sc->n_tris; done_linear = 1;
        } else {
            if (!sp) break;
            const or_node* nd = sc->nodes + st[--sp];
            if (!box_hit(nd, o, d, INFINITY)) continue;
            if (nd->left >= 0) { st[sp++] = nd->right; st[sp++] = nd->left; continue; }
            first = nd->first; count = nd->count;
        }
        for (int64_t q = first; q < first + count; ++q) {
            int64_t tid = sc->use_bvh ? sc->perm[q] : q;
            const float* v = sc->tv + 9 * tid;
            or_tri_res r;
            watertight(o, d, &s, v, v + 3, v + 6, &r);
            if (r.hit) {
                hit = 1;
                if (r.margin >= OR_TIE) { robust = 1; break; }
                near = 1;
            } else if (r.margin < OR_TIE && r.t_pos) {
                near = 1;
            }
        }
    }
    free(big);
    *flag = (!robust && near) ? 1 : 0;
    return hit;
}

/* Public closest-hit / any-hit over ray arrays (OpenMP over rays). */
void or_trace_closest(const or_scene* sc, int64_t n, const float* org, const float* dir, int32_t* id, float* t,
                      uint8_t* flag) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        or_closest c;
        uint8_t f;
        closest(sc, org + 3 * i, dir + 3 * i, &c, &f);
        id[i] = c.id;
        t[i] = c.id >= 0 ? c.t : INFINITY;
        if (flag) flag[i] = f;
    }
}

/* occluded = 1 iff some triangle is hit with t > 0 (edges included, as the
 * watertight test decides them); near-edge-only cases are flagged. */
void or_trace_any(const or_scene* sc, int64_t n, const float* org, const float* dir, uint8_t* occluded,
                  uint8_t* flag) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        uint8_t f;
        occluded[i] = (uint8_t)anyhit(sc, org + 3 * i, dir + 3 * i, &f);
        if (flag) flag[i] = f;
    }
}

/* ------------------------------------------------------------------------ */
/* Shading (Sec. 6.1: closest-hit shading, miss shader)                      */
/* ------------------------------------------------------------------------ */

/* 32-bit integer hash: the PCG-based hash of Jarzynski and Olano, "Hash
 * Functions for GPU Rendering", JCGT 9(3), 2020. */
static uint32_t pcg_hash(uint32_t v) {
    uint32_t state = v * 747796405u + 2891336453u;
    uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}

/* Per-triangle albedo: 0.2 + 0.7 x (one byte of the hash) / 255 per channel. */
static void albedo(int32_t id, float* a) {
    uint32_t h = pcg_hash((uint32_t)id);
    a[0] = 0.2f + 0.7f * (float)(h & 255u) / 255.0f;
    a[1] = 0.2f + 0.7f * (float)((h >> 8) & 255u) / 255.0f;
    a[2] = 0.2f + 0.7f * (float)((h >> 16) & 255u) / 255.0f;
}

void or_albedo_many(int64_t n, const int32_t* id, float* rgb) {
    for (int64_t i = 0; i < n; ++i) albedo(id[i], rgb + 3 * i);
}

/*
 * Geometric normal and shadow-ray origin, FP32, each rounding stated:
 *   e1 = v1 - v0, e2 = v2 - v0, n = e1 x e2 (plain products and differences)
 *   len = sqrt((nx nx + ny ny) + nz nz); n = n / len when len > 0
 *   n is negated when (nx dx + ny dy) + nz dz > 0 (it faces the ray)
 *   p = fma(t, d, o); eps = 1e-4 (1 + max |p_k|); o_s = fma(eps, n, p)
 */
static void hit_frame(const float* v, const float* o, const float* d, float t, float* n, float* p, float* os) {
    float e1[3], e2[3];
    for (int k = 0; k < 3; ++k) { e1[k] = v[3 + k] - v[k]; e2[k] = v[6 + k] - v[k]; }
    float a, b;
    a = e1[1] * e2[2]; b = e1[2] * e2[1]; n[0] = a - b;
    a = e1[2] * e2[0]; b = e1[0] * e2[2]; n[1] = a - b;
    a = e1[0] * e2[1]; b = e1[1] * e2[0]; n[2] = a - b;
    float l2 = (n[0] * n[0] + n[1] * n[1]) + n[2] * n[2];
    float len = sqrtf(l2);
    if (len > 0.0f) { n[0] = n[0] / len; n[1] = n[1] / len; n[2] = n[2] / len; }
    float nd = (n[0] * d[0] + n[1] * d[1]) + n[2] * d[2];
    if (nd > 0.0f) { n[0] = -n[0]; n[1] = -n[1]; n[2] = -n[2]; }
    float mx = 0.0f;
    for (int k = 0; k < 3; ++k) {
        p[k] = fmaf(t, d[k], o[k]);
        float ap = fabsf(p[k]);
        if (ap > mx) mx = ap;
    }
    float eps = 1e-4f * (1.0f + mx);
    for (int k = 0; k < 3; ++k) os[k] = fmaf(eps, n[k], p[k]);
}

/*
 * Lambert shading with one directional light and one shadow ray.
 * sh = {light_dir[3] (unit, toward the light), light_rgb[3], ambient[3],
 *       background[3], shadow (0/1)}.
 * miss -> background; hit -> albedo (ambient + light max(0, n.l) vis), where
 * vis = 0 iff the shadow ray from o_s along light_dir hits anything with
 * t > 0.  The shadow ray is cast only when n.l > 0 (otherwise vis has no
 * effect).  Alpha is 1.  rgba is FP32 linear, no tone map.
 */
void or_shade_rays(const or_scene* sc, int64_t n, const float* org, const float* dir, const float* sh,
                   float* rgba, int32_t* id_out, uint8_t* flag_out) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        const float* o = org + 3 * i;
        const float* d = dir + 3 * i;
        or_closest c;
        uint8_t f = 0;
        closest(sc, o, d, &c, &f);
        float* out = rgba + 4 * i;
        if (c.id < 0) {
            out[0] = sh[9]; out[1] = sh[10]; out[2] = sh[11]; out[3] = 1.0f;
        } else {
            const float* v = sc->tv + 9 * (int64_t)c.id;
            float nrm[3], p[3], os[3], alb[3];
            hit_frame(v, o, d, c.t, nrm, p, os);
            albedo(c.id, alb);
            float ndl = (nrm[0] * sh[0] + nrm[1] * sh[1]) + nrm[2] * sh[2];
            float vis = 1.0f;
            if (ndl > 0.0f && sh[12] != 0.0f) {
                uint8_t sf = 0;
                if (anyhit(sc, os, sh, &sf)) vis = 0.0f;
                if (sf) f = 1;
            }
            float lam = ndl > 0.0f ? ndl : 0.0f;
            for (int k = 0; k < 3; ++k) out[k] = alb[k] * (sh[6 + k] + sh[3 + k] * lam * vis);
            out[3] = 1.0f;
        }
        if (id_out) id_out[i] = c.id;
        if (flag_out) flag_out[i] = f;
    }
}

/* ------------------------------------------------------------------------ */
/* Path-traced LP shading (Sec. 8: one sample per LP texel)                  */
/* ------------------------------------------------------------------------ */

/*
 * Counter-based random numbers: u32 = pcg_hash chained over the key words
 * (seed_lo, seed_hi, frame, view, texel, bounce*8 + dim); the float is the top
 * 24 bits times 2^-24.
 */
static float rng01(uint32_t seed_lo, uint32_t seed_hi, uint32_t frame, uint32_t view, uint32_t texel,
                   uint32_t slot) {
    uint32_t h = pcg_hash(seed_lo);
    h = pcg_hash(h ^ seed_hi);
    h = pcg_hash(h ^ frame);
    h = pcg_hash(h ^ view);
    h = pcg_hash(h ^ texel);
    h = pcg_hash(h ^ slot);
    return (float)(h >> 8) * (1.0f / 16777216.0f);
}

float or_rng01(uint64_t seed, uint32_t frame, uint32_t view, uint32_t texel, uint32_t slot) {
    return rng01((uint32_t)seed, (uint32_t)(seed >> 32), frame, view, texel, slot);
}

/*
 * Cosine-weighted direction about the unit normal n (Malley's method: a
 * uniform point of the unit disk lifted to the hemisphere).  The disk point
 * comes from rejection sampling of the square with up to 8 tries, each try
 * using two fresh random slots; after 8 rejections the centre is used.  The
 * tangent frame is that of Duff et al., "Building an Orthonormal Basis,
 * Revisited", JCGT 6(1), 2017.  FP32, each rounding stated:
 *   x = 2 r0 - 1, y = 2 r1 - 1, accept when (x x + y y) < 1
 *   z = sqrt(max(0, (1 - x x) - y y))
 *   s = copysign(1, nz), a = -1 / (s + nz), b = nx ny a
 *   t1 = (1 + s nx nx a, s b, -s nx), t2 = (b, s + ny ny a, -ny)
 *   w = (x t1 + y t2) + z n, per component with plain products and sums
 */
static void cosine_dir(const float* n, uint32_t slo, uint32_t shi, uint32_t frame, uint32_t view, uint32_t texel,
                       uint32_t bounce, float* w) {
    float x = 0.0f, y = 0.0f;
    for (uint32_t tr = 0; tr < 8; ++tr) {
        float r0 = rng01(slo, shi, frame, view, texel, bounce * 32u + 2u * tr + 0u);
        float r1 = rng01(slo, shi, frame, view, texel, bounce * 32u + 2u * tr + 1u);
        float xx = 2.0f * r0 - 1.0f, yy = 2.0f * r1 - 1.0f;
        float q = xx * xx + yy * yy;
        if (q < 1.0f) { x = xx; y = yy; break; }
    }
    float zz = (1.0f - x * x) - y * y;
    float z = sqrtf(zz > 0.0f ? zz : 0.0f);
    float s = copysignf(1.0f, n[2]);
    float a = -1.0f / (s + n[2]);
    float b = n[0] * n[1] * a;
    float t1[3] = {1.0f + s * n[0] * n[0] * a, s * b, -s * n[0]};
    float t2[3] = {b, s + n[1] * n[1] * a, -n[1]};
    for (int k = 0; k < 3; ++k) {
        float p1 = x * t1[k];
        float p2 = y * t2[k];
        float p3 = z * n[k];
        w[k] = (p1 + p2) + p3;
    }
}

/*
 * One path sample per ray: at every vertex, next-event estimation toward the
 * directional light (shadow ray) and a cosine-weighted continuation, up to
 * `bounces` continuation rays (bounces = 2: the primary hit plus two more
 * vertices).  Throughput is multiplied by the albedo at each vertex (the
 * cosine-weighted pdf cancels the Lambert cosine).  A continuation ray that
 * misses adds throughput x background (sky light).  No Russian roulette.
 * pt = {seed (u64), frame, view, bounces}; texel ids are idx[].
 */
void or_shade_path_rays(const or_scene* sc, int64_t n, const float* org, const float* dir, const int64_t* idx,
                        const float* sh, uint64_t seed, uint32_t frame, uint32_t view, int32_t bounces,
                        float* rgba, int32_t* id_out, uint8_t* flag_out) {
    uint32_t slo = (uint32_t)seed, shi = (uint32_t)(seed >> 32);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        float o[3] = {org[3 * i], org[3 * i + 1], org[3 * i + 2]};
        float d[3] = {dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]};
        float thr[3] = {1.0f, 1.0f, 1.0f};
        float L[3] = {0.0f, 0.0f, 0.0f};
        uint8_t f = 0;
        int32_t first_id = -1;
        uint32_t texel = (uint32_t)idx[i];
        for (int32_t bnc = 0; bnc <= bounces; ++bnc) {
            or_closest c;
            uint8_t cf = 0;
            closest(sc, o, d, &c, &cf);
            if (cf) f = 1;
            if (bnc == 0) first_id = c.id;
            if (c.id < 0) {
                for (int k = 0; k < 3; ++k) L[k] += thr[k] * sh[9 + k];
                break;
            }
            const float* v = sc->tv + 9 * (int64_t)c.id;
            float nrm[3], p[3], os[3], alb[3];
            hit_frame(v, o, d, c.t, nrm, p, os);
            albedo(c.id, alb);
            float ndl = (nrm[0] * sh[0] + nrm[1] * sh[1]) + nrm[2] * sh[2];
            float vis = 0.0f;
            if (ndl > 0.0f) {
                uint8_t sf = 0;
                vis = anyhit(sc, os, sh, &sf) ? 0.0f : 1.0f;
                if (sf) f = 1;
            }
            for (int k = 0; k < 3; ++k) {
                thr[k] = thr[k] * alb[k];
                L[k] += thr[k] * (sh[6 + k] + sh[3 + k] * ndl * vis);
            }
            if (bnc == bounces) break;
            float w[3];
            cosine_dir(nrm, slo, shi, frame, view, texel, (uint32_t)bnc, w);
            for (int k = 0; k < 3; ++k) { o[k] = os[k]; d[k] = w[k]; }
        }
        float* out = rgba + 4 * i;
        out[0] = L[0]; out[1] = L[1]; out[2] = L[2]; out[3] = 1.0f;
        if (id_out) id_out[i] = first_id;
        if (flag_out) flag_out[i] = f;
    }
}

/* ------------------------------------------------------------------------ */
/* Inverse mapping / reconstruction (Sec. 3.2.3, Eqs. (10)-(11))             */
/* ------------------------------------------------------------------------ */

static double fmod_pos(double a, double m) {
    double r = fmod(a, m);
    return r < 0.0 ? r + m : r;
}

/*
 * Each display pixel centre is forward-mapped to (u, theta) (Eqs. (3), (5)),
 * and the LP buffer is sampled there (the paper's inverse-mapping pass; its
 * filter is not stated).  Filter: u is clamped to [1/2, N_c - 1/2]; the two
 * columns around u - 1/2 are blended linearly; inside each column the two
 * rows around theta/360 n_i - 1/2 are blended linearly with wrap-around in
 * theta (rows tile the circle), which keeps the filter continuous in angle
 * although neighbouring columns hold different row counts.
 * pflag (optional) marks pixels that read a texel whose tflag is set.
 */
/* Sampling positions of display pixel `pix`: per side (0: column i0, 1:
 * column i1) the texels k[side][0..1] of the two rows around the pixel's
 * angle, the row weight tt[side], and the column weight wc of side 1. */
static void vafr_pixel_taps(const or_acuity* a, int32_t n_cols, const int32_t* n_rows, const int64_t* col_off,
                            int32_t W, int32_t H, const double* p, const double* G, int64_t pix, int64_t k[2][2],
                            double tt[2], double* wc_out) {
    int64_t x = pix % W, y = pix / W;
    double X = ((double)x + 0.5 - 0.5 * W) * p[0];
    double Y = ((double)y + 0.5 - 0.5 * H) * p[1];
    double dx = X - G[0], dy = Y - G[1];
    double rho = sqrt(dx * dx + dy * dy);
    double e = atan(rho) / OR_DEG;
    double th = atan2(dy, dx) / OR_DEG;
    if (th < 0.0) th += 360.0;
    double u = or_u(a, e);
    if (u < 0.5) u = 0.5;
    if (u > n_cols - 0.5) u = n_cols - 0.5;
    double ac = u - 0.5;
    int64_t i0 = (int64_t)floor(ac);
    if (i0 > n_cols - 1) i0 = n_cols - 1;
    int64_t i1 = i0 + 1 < n_cols ? i0 + 1 : n_cols - 1;
    *wc_out = ac - (double)i0;
    for (int side = 0; side < 2; ++side) {
        int64_t i = side ? i1 : i0;
        int64_t ni = n_rows[i];
        double s = th / 360.0 * (double)ni - 0.5;
        double fs = floor(s);
        tt[side] = s - fs;
        int64_t j0 = (int64_t)fmod_pos(fs, (double)ni);
        int64_t j1 = (j0 + 1) % ni;
        k[side][0] = col_off[i] + j0;
        k[side][1] = col_off[i] + j1;
    }
}

void or_vafr_reconstruct(const or_acuity* a, int32_t n_cols, const int32_t* n_rows, const int64_t* col_off,
                         const float* lp, int32_t W, int32_t H, const double* p, const double* G,
                         const int64_t* pix, int64_t n, float* out, const uint8_t* tflag, uint8_t* pflag) {
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) {
        int64_t k[2][2];
        double tt[2], wc;
        vafr_pixel_taps(a, n_cols, n_rows, col_off, W, H, p, G, pix[q], k, tt, &wc);
        double acc[4] = {0, 0, 0, 0};
        uint8_t fl = 0;
        for (int side = 0; side < 2; ++side) {
            double wi = side ? wc : 1.0 - wc;
            int64_t k0 = k[side][0], k1 = k[side][1];
            for (int ch = 0; ch < 4; ++ch)
                acc[ch] += wi * ((1.0 - tt[side]) * (double)lp[4 * k0 + ch] + tt[side] * (double)lp[4 * k1 + ch]);
            if (tflag && (tflag[k0] || tflag[k1])) fl = 1;
        }
        for (int ch = 0; ch < 4; ++ch) out[4 * q + ch] = (float)acc[ch];
        if (pflag) pflag[q] = fl;
    }
}

/* The four texels display pixel pix[q] reads: taps[4 q ..] = column i0's
 * two rows, then column i1's (test infrastructure: reconstruction
 * footprints). */
void or_vafr_taps(const or_acuity* a, int32_t n_cols, const int32_t* n_rows, const int64_t* col_off, int32_t W,
                  int32_t H, const double* p, const double* G, const int64_t* pix, int64_t n, int64_t* taps) {
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) {
        int64_t k[2][2];
        double tt[2], wc;
        vafr_pixel_taps(a, n_cols, n_rows, col_off, W, H, p, G, pix[q], k, tt, &wc);
        taps[4 * q] = k[0][0];
        taps[4 * q + 1] = k[0][1];
        taps[4 * q + 2] = k[1][0];
        taps[4 * q + 3] = k[1][1];
    }
}

/*
 * Bilinear sample of a dense w x h log-polar buffer (k = i h + j) at column
 * coordinate u and row coordinate v (texel centres at + 1/2): u clamped to
 * the first / last column centre, v wrapping.  fl is set when one of the
 * four texels is flagged in tflag.
 */
static void dense_sample(int32_t w, int32_t h, const float* lp, double u, double v, const uint8_t* tflag,
                         float* out, uint8_t* fl) {
    if (u < 0.5) u = 0.5;
    if (u > w - 0.5) u = w - 0.5;
    double ac = u - 0.5;
    int64_t i0 = (int64_t)floor(ac);
    if (i0 > w - 1) i0 = w - 1;
    int64_t i1 = i0 + 1 < w ? i0 + 1 : w - 1;
    double wc = ac - (double)i0;
    double s = v - 0.5;
    double fs = floor(s);
    double tt = s - fs;
    int64_t j0 = (int64_t)fmod_pos(fs, (double)h);
    int64_t j1 = (j0 + 1) % h;
    double acc[4] = {0, 0, 0, 0};
    *fl = 0;
    int64_t ks[4] = {i0 * h + j0, i0 * h + j1, i1 * h + j0, i1 * h + j1};
    double ws[4] = {(1 - wc) * (1 - tt), (1 - wc) * tt, wc * (1 - tt), wc * tt};
    for (int c = 0; c < 4; ++c) {
        for (int ch = 0; ch < 4; ++ch) acc[ch] += ws[c] * (double)lp[4 * ks[c] + ch];
        if (tflag && tflag[ks[c]]) *fl = 1;
    }
    for (int ch = 0; ch < 4; ++ch) out[ch] = (float)acc[ch];
}

/*
 * LMFR reconstruction: the pixel centre maps through Eq. (1) with K(z) =
 * z^alpha to (u, v); the dense w x h buffer is sampled bilinearly at
 * (u - 1/2, v - 1/2), clamped in u and wrapped in v.
 */
void or_lmfr_reconstruct(int32_t W, int32_t H, double gx, double gy, int32_t w, int32_t h, double alpha,
                         const float* lp, const int64_t* pix, int64_t n, float* out, const uint8_t* tflag,
                         uint8_t* pflag) {
    double L = or_lmfr_L(W, H, gx, gy);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) {
        int64_t x = pix[q] % W, y = pix[q] / W;
        double dx = (double)x + 0.5 - gx, dy = (double)y + 0.5 - gy;
        double r = sqrt(dx * dx + dy * dy);
        if (r < 1.0) r = 1.0;
        double z = log(r) / L;
        double th = atan2(dy, dx) / OR_DEG;
        if (th < 0.0) th += 360.0;
        uint8_t fl;
        dense_sample(w, h, lp, pow(z, alpha) * w, th / 360.0 * h, tflag, out + 4 * q, &fl);
        if (pflag) pflag[q] = fl;
    }
}

/* LaFR reconstruction: as LMFR with the map of Eq. (15).  Returns
 * or_lafr_consts' status. */
int or_lafr_reconstruct(int32_t W, int32_t H, const double* p, double gx, double gy, int32_t w, int32_t h,
                        double a, double alpha, double beta, const float* lp, const int64_t* pix, int64_t n,
                        float* out, const uint8_t* tflag, uint8_t* pflag) {
    double c[4];
    if (or_lafr_consts(W, H, p, gx, gy, a, alpha, c)) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) {
        int64_t x = pix[q] % W, y = pix[q] / W;
        double dx = (double)x + 0.5 - gx, dy = (double)y + 0.5 - gy;
        double r = sqrt(dx * dx + dy * dy);
        if (r < 1.0) r = 1.0;
        double z = log(r) / c[0];
        double th = atan2(dy, dx) / OR_DEG;
        if (th < 0.0) th += 360.0;
        uint8_t fl;
        dense_sample(w, h, lp, lafr_u(c, beta, z) * w, th / 360.0 * h, tflag, out + 4 * q, &fl);
        if (pflag) pflag[q] = fl;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* FXAA-style edge anti-aliasing inside the LP buffer (Sec. 3.4)            */
/* ------------------------------------------------------------------------ */

/*
 * The paper runs FXAA (Lottes, "FXAA", NVIDIA white paper 2009) on the LP
 * buffer and gives no further detail.  On the ragged polar grid the steps
 * of that method are taken as follows (every operation in FP32, in the order
 * written, so that the library's kernel can agree bit for bit):
 *
 *  - a texel's neighbours along the angle are the adjacent rows of its own
 *    column (cyclic); its neighbours along the radius are the inner and
 *    outer columns sampled at the texel's angle, linear in the row
 *    coordinate; diagonal neighbours are those columns at the angle one row
 *    (of the texel's column) before and after.  Columns clamp at the ends.
 *  - luma = 0.299 r + 0.587 g + 0.114 b.
 *  - contrast test: the texel is left unchanged when the luma range over
 *    itself and its four direct neighbours is below
 *    max(FXAA_EDGE_MIN, FXAA_EDGE_REL * max luma).
 *  - orientation: second differences of luma across the radius (summed over
 *    the three angles, centre weighted 2) against those across the angle;
 *    the larger decides the edge normal.
 *  - the side of the edge is the neighbour along the normal with the larger
 *    luma step; the edge line lies midway between the texel and that side.
 *  - end search: along the edge line in both directions at offsets
 *    FXAA_STEPS (in rows of the texel's column, or in columns), sampling the
 *    mean luma of the two sides of the line, until it differs from the
 *    line's mean at the texel by at least a quarter of the luma step;
 *    an end not found is taken one step beyond the last offset.
 *  - edge blend: 0.5 - d_near / (d_neg + d_pos) when the nearer end
 *    continues the texel's side of the edge, else 0.
 *  - sub-texel blend: smoothstep of |mean of neighbours - centre| / range
 *    (direct neighbours weighted 2, diagonals 1, over 12), squared, times
 *    FXAA_SUBPIX.
 *  - output: centre + max(edge blend, sub-texel blend) x (side value -
 *    centre), per channel.
 */
#define FXAA_EDGE_REL 0.125f
#define FXAA_EDGE_MIN 0.0625f
#define FXAA_SUBPIX 0.75f
#define FXAA_NSTEP 6
static const float FXAA_STEPS[FXAA_NSTEP] = {1.0f, 2.0f, 3.0f, 4.0f, 6.0f, 8.0f};

typedef struct { float v[4]; } or_px;

typedef struct {
    int32_t n_cols;
    const int32_t* n_rows;
    const int64_t* col_off;
    const float* lp;
} or_lpgrid;

static or_px fx_tex(const or_lpgrid* g, int32_t c, int64_t j) {
    int64_t n = g->n_rows[c];
    int64_t jj = j % n;
    if (jj < 0) jj += n;
    or_px p;
    for (int k = 0; k < 4; ++k) p.v[k] = g->lp[4 * (g->col_off[c] + jj) + k];
    return p;
}

static int32_t fx_clamp_col(const or_lpgrid* g, int32_t c) { return c < 0 ? 0 : (c >= g->n_cols ? g->n_cols - 1 : c); }

/* Column c at angle t turns: linear between the rows around t n - 1/2. */
static or_px fx_col(const or_lpgrid* g, int32_t c, float t) {
    c = fx_clamp_col(g, c);
    float s = t * (float)g->n_rows[c] - 0.5f;
    float fs = floorf(s);
    float w = s - fs;
    int64_t j0 = (int64_t)fs;
    or_px a = fx_tex(g, c, j0), b = fx_tex(g, c, j0 + 1), r;
    for (int k = 0; k < 4; ++k) {
        float d = b.v[k] - a.v[k];
        r.v[k] = a.v[k] + w * d;
    }
    return r;
}

static float fx_luma(or_px p) {
    float a = 0.299f * p.v[0];
    float b = 0.587f * p.v[1];
    float c = 0.114f * p.v[2];
    return (a + b) + c;
}

static float fx_second(float a, float m, float b) {
    float d = (a - m) + (b - m);
    return fabsf(d);
}

static or_px fx_texel(const or_lpgrid* g, int32_t i, int32_t j) {
    const int32_t n = g->n_rows[i];
    const float t = ((float)j + 0.5f) / (float)n;
    const float dt = 1.0f / (float)n;
    const or_px M = fx_tex(g, i, j);
    const float lM = fx_luma(M);
    const float lU = fx_luma(fx_tex(g, i, (int64_t)j + 1));
    const float lD = fx_luma(fx_tex(g, i, (int64_t)j - 1));
    const or_px O = fx_col(g, i + 1, t), I = fx_col(g, i - 1, t);
    const float lO = fx_luma(O), lI = fx_luma(I);
    float lmax = fmaxf(fmaxf(fmaxf(lM, lU), fmaxf(lD, lO)), lI);
    float lmin = fminf(fminf(fminf(lM, lU), fminf(lD, lO)), lI);
    const float range = lmax - lmin;
    if (range < fmaxf(FXAA_EDGE_MIN, lmax * FXAA_EDGE_REL)) return M;
    const float lOU = fx_luma(fx_col(g, i + 1, t + dt)), lOD = fx_luma(fx_col(g, i + 1, t - dt));
    const float lIU = fx_luma(fx_col(g, i - 1, t + dt)), lID = fx_luma(fx_col(g, i - 1, t - dt));
    /* second differences across the radius (at three angles) and across the
     * angle (at three radii) */
    const float eR = (fx_second(lID, lD, lOD) + 2.0f * fx_second(lI, lM, lO)) + fx_second(lIU, lU, lOU);
    const float eA = (fx_second(lID, lI, lIU) + 2.0f * fx_second(lD, lM, lU)) + fx_second(lOD, lO, lOU);
    const int normal_radial = eR >= eA; /* luma changes across the radius: the edge runs along the angle */
    const float lNeg = normal_radial ? lI : lD, lPos = normal_radial ? lO : lU;
    const float gNeg = fabsf(lNeg - lM), gPos = fabsf(lPos - lM);
    const int side = gPos >= gNeg ? 1 : -1;
    const float lSide = side > 0 ? lPos : lNeg;
    const float grad = fmaxf(gNeg, gPos);
    const float lLine = 0.5f * (lM + lSide);
    const float gScaled = 0.25f * grad;
    float dist[2];
    float lEnd[2];
    for (int dir = 0; dir < 2; ++dir) {
        const float sgn = dir == 0 ? -1.0f : 1.0f;
        dist[dir] = FXAA_STEPS[FXAA_NSTEP - 1] + 1.0f;
        lEnd[dir] = lLine;
        for (int k = 0; k < FXAA_NSTEP; ++k) {
            const float p = sgn * FXAA_STEPS[k];
            float la, lb;
            if (normal_radial) {
                /* along the angle, between column i and column i + side */
                const float tt = t + p * dt;
                la = fx_luma(fx_col(g, i, tt));
                lb = fx_luma(fx_col(g, i + side, tt));
            } else {
                /* along the radius, between angle t and t + side dt */
                const int32_t c = i + (int32_t)p;
                la = fx_luma(fx_col(g, c, t));
                lb = fx_luma(fx_col(g, c, t + (float)side * dt));
            }
            const float l = 0.5f * (la + lb);
            if (fabsf(l - lLine) >= gScaled) {
                dist[dir] = FXAA_STEPS[k];
                lEnd[dir] = l;
                break;
            }
        }
    }
    const int near = dist[0] <= dist[1] ? 0 : 1;
    const float dNear = dist[near];
    const int centre_below = lM - lLine < 0.0f;
    const int end_below = lEnd[near] - lLine < 0.0f;
    const float edge = centre_below != end_below ? 0.5f - dNear / (dist[0] + dist[1]) : 0.0f;
    const float lAvg = (2.0f * ((lU + lD) + (lI + lO)) + ((lIU + lID) + (lOU + lOD))) / 12.0f;
    float s1 = fabsf(lAvg - lM) / range;
    s1 = fminf(fmaxf(s1, 0.0f), 1.0f);
    const float s2 = (-2.0f * s1 + 3.0f) * (s1 * s1);
    const float sub = (s2 * s2) * FXAA_SUBPIX;
    const float off = fmaxf(edge, sub);
    or_px S = normal_radial ? fx_col(g, i + side, t) : fx_tex(g, i, (int64_t)j + side);
    or_px r;
    for (int k = 0; k < 4; ++k) {
        float d = S.v[k] - M.v[k];
        r.v[k] = M.v[k] + off * d;
    }
    return r;
}

/* FXAA over texels idx[0..n) of the LP buffer; out holds 4 floats per
 * listed texel. */
void or_fxaa_lp(int32_t n_cols, const int32_t* n_rows, const int64_t* col_off, const float* lp, const int64_t* idx,
                int64_t n, float* out) {
    or_lpgrid g = {n_cols, n_rows, col_off, lp};
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; ++q) {
        int64_t k = idx[q];
        /* column of texel k */
        int32_t lo = 0, hi = n_cols - 1;
        while (lo < hi) {
            int32_t mid = (lo + hi + 1) / 2;
            if (col_off[mid] <= k) lo = mid;
            else hi = mid - 1;
        }
        or_px r = fx_texel(&g, lo, (int32_t)(k - col_off[lo]));
        for (int c = 0; c < 4; ++c) out[4 * q + c] = r.v[c];
    }
}
/* ------------------------------------------------------------------------ */
/* Binocular reprojection by forward grid warping of the left LP buffer     */
/* (VaFR_Rep, Sec. 5.1)                                                     */
/* ------------------------------------------------------------------------ */

/*
 * The paper renders the right eye by warping the left eye's LP buffer as a
 * grid (forward grid warping after Wissmann et al. 2020) instead of
 * rendering it again.  For ray casting this is taken as follows.
 *
 * Vertices.  Every left texel whose primary ray hits carries its hit point
 * p = fma(t, d, o) (FP32, as the hit frame forms it).  Projected into the
 * right eye (FP32, in this order): q = p - eye_R; x = q.R, y = q.U,
 * z = q.F, each dot product summed left to right; film point
 * (x / z, -(y / z)).  A vertex is valid when its ray hit, z > 0 and the
 * film point is finite.
 *
 * Grid.  Texel (i, j) of column i (n_i rows) sits at angle (2j + 1) / (2 n_i)
 * turns.  The band between columns s and s + 1 is triangulated by a zipper
 * walk: the texels of both columns are merged by angle (on equal angles the
 * inner column first), cyclically; each texel x met in that order closes
 * the triangle (previous texel of x's column, x, last texel of the other
 * column met before x -- the other column's last texel when none was).
 * Triangle ids: 2 x + 1 for x in the inner column of the band, 2 x for x in
 * the outer column.
 *
 * Discarded triangles (their area is left to ray casting): a vertex not
 * valid; a depth jump, largest z > (1 + 1/10) x smallest z; a stretch, the
 * right film bounding box's larger side above twice the larger side of the
 * left film bounding box of the same texels; zero area.
 *
 * Coverage (FP64).  Right texel c's sample point is C = G + dxy[c] (the
 * gaze film point plus its film offset, as its primary ray uses).  With
 * E(P, Q; C) = (Q.x - P.x)(C.y - P.y) - (Q.y - P.y)(C.x - P.x), vertices
 * V0 = previous, V1 = x, V2 = other, A = E(V0, V1; V2), e0 = E(V1, V2; C),
 * e1 = E(V2, V0; C), e2 = E(V0, V1; C): C is covered when A != 0 and every
 * e_k has A's sign or is zero.  b_k = e_k / A, s = b0/z0 + b1/z1 + b2/z2,
 * depth = (float)(1 / s) (perspective-correct: 1/z is linear on the film).
 * The covering triangle of least (depth bits, id) wins the texel.
 *
 * Colour.  w_k = (b_k / z_k) / s; rgba = w0 c0 + w1 c1 + w2 c2 (FP64, left to
 * right, rounded to FP32); hit id of the vertex of largest w (first on
 * ties).  Right texels no triangle covers are ray cast as usual.
 *
 * This function is the plain definition: the triangles are listed by the
 * zipper walk and every texel is tested against the triangles of its bin on
 * a uniform grid over the right film plane (no log-polar geometry).
 *
 * flag marks right texels whose result may legitimately differ: those whose
 * sample point lies in the bounding box, widened by its size on every
 * side, of the valid vertices of a triangle that uses a flagged left texel
 * (near-tie hit, which another FP32 implementation may resolve to the other
 * triangle).  tri[c] = winning triangle id or -1; depth_win[c] (nullable)
 * its depth.
 */
#define OR_WARP_DEPTH_REL 0.1
#define OR_WARP_STRETCH 2.0

typedef struct {
    int64_t v[3];      /* texels: previous, x, other */
    int64_t id;
} or_wtri;

/* zipper walk of the band between columns s and s + 1; appends its
 * triangles to out (2 n_s + 2 n_{s+1} entries reserved by the caller). */
static int64_t warp_band(const int32_t* n_rows, const int64_t* col_off, int32_t s, or_wtri* out) {
    const int64_t na = n_rows[s], nb = n_rows[s + 1];
    const int64_t oa = col_off[s], ob = col_off[s + 1];
    int64_t ka = 0, kb = 0, m = 0;
    int64_t last_a = -1, last_b = -1;   /* last texel met in each column */
    while (ka < na || kb < nb) {
        int take_a;
        if (ka >= na) take_a = 0;
        else if (kb >= nb) take_a = 1;
        else take_a = (2 * ka + 1) * nb <= (2 * kb + 1) * na;   /* inner first on ties */
        if (take_a) {
            const int64_t x = oa + ka;
            out[m].v[0] = oa + (ka == 0 ? na - 1 : ka - 1);
            out[m].v[1] = x;
            out[m].v[2] = last_b >= 0 ? last_b : ob + nb - 1;
            out[m].id = 2 * x + 1;
            last_a = x;
            ++ka;
        } else {
            const int64_t x = ob + kb;
            out[m].v[0] = ob + (kb == 0 ? nb - 1 : kb - 1);
            out[m].v[1] = x;
            out[m].v[2] = last_a >= 0 ? last_a : oa + na - 1;
            out[m].id = 2 * x;
            last_b = x;
            ++kb;
        }
        ++m;
    }
    return m;
}

/* All grid triangles, ordered by band; returns their number (the caller
 * frees *tris). */
int64_t or_warp_triangles(int32_t n_cols, const int32_t* n_rows, const int64_t* col_off, int64_t* tri_v,
                          int64_t* tri_id) {
    const int64_t n = col_off[n_cols];
    or_wtri* t = (or_wtri*)malloc(sizeof(or_wtri) * (size_t)(2 * n + 1));
    int64_t m = 0;
    for (int32_t s = 0; s + 1 < n_cols; ++s) m += warp_band(n_rows, col_off, s, t + m);
    if (tri_v)
        for (int64_t k = 0; k < m; ++k) {
            for (int c = 0; c < 3; ++c) tri_v[3 * k + c] = t[k].v[c];
            tri_id[k] = t[k].id;
        }
    free(t);
    return m;
}

static double warp_edge(const double* P, const double* Q, const double* Cp) {
    return (Q[0] - P[0]) * (Cp[1] - P[1]) - (Q[1] - P[1]) * (Cp[0] - P[0]);
}

void or_rep_warp(int32_t n_cols, const int32_t* n_rows, const int64_t* col_off, const float* dxy, const double* G,
                 const float* org, const float* dir, const float* t, const int32_t* hit_id, const uint8_t* lflag,
                 const float* rgba_left, const float* cam_right, float* rgba_right, int32_t* id_right,
                 int64_t* tri_win, float* depth_win, uint8_t* flag) {
    const int64_t n = col_off[n_cols];
    const float* eye = cam_right;
    const float* R = cam_right + 3;
    const float* U = cam_right + 6;
    const float* F = cam_right + 9;
    /* vertices: right film point and depth */
    double* fp = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    float* zr = (float*)malloc(sizeof(float) * (size_t)n);
    uint8_t* ok = (uint8_t*)malloc((size_t)n);
    for (int64_t k = 0; k < n; ++k) {
        ok[k] = 0;
        if (hit_id[k] < 0) continue;
        float p[3], q[3];
        for (int c = 0; c < 3; ++c) {
            p[c] = fmaf(t[k], dir[3 * k + c], org[3 * k + c]);
            q[c] = p[c] - eye[c];
        }
        float x = (q[0] * R[0] + q[1] * R[1]) + q[2] * R[2];
        float y = (q[0] * U[0] + q[1] * U[1]) + q[2] * U[2];
        float z = (q[0] * F[0] + q[1] * F[1]) + q[2] * F[2];
        if (!(z > 0.0f)) continue;
        float fx = x / z, fy = -(y / z);
        if (!isfinite(fx) || !isfinite(fy)) continue;
        fp[2 * k] = fx;
        fp[2 * k + 1] = fy;
        zr[k] = z;
        ok[k] = 1;
    }
    /* triangles, kept ones with their right film boxes */
    int64_t* tv = (int64_t*)malloc(sizeof(int64_t) * 3 * (size_t)(2 * n + 1));
    int64_t* tid = (int64_t*)malloc(sizeof(int64_t) * (size_t)(2 * n + 1));
    const int64_t m = or_warp_triangles(n_cols, n_rows, col_off, tv, tid);
    uint8_t* keep = (uint8_t*)calloc((size_t)m, 1);
    double* box = (double*)malloc(sizeof(double) * 4 * (size_t)m);   /* x0 y0 x1 y1 */
    double gx0 = INFINITY, gy0 = INFINITY, gx1 = -INFINITY, gy1 = -INFINITY;
    for (int64_t k = 0; k < m; ++k) {
        const int64_t* v = tv + 3 * k;
        if (!ok[v[0]] || !ok[v[1]] || !ok[v[2]]) continue;
        float zmin = zr[v[0]], zmax = zr[v[0]];
        for (int c = 1; c < 3; ++c) {
            zmin = zr[v[c]] < zmin ? zr[v[c]] : zmin;
            zmax = zr[v[c]] > zmax ? zr[v[c]] : zmax;
        }
        if ((double)zmax > (double)zmin * (1.0 + OR_WARP_DEPTH_REL)) continue;
        double rx0 = INFINITY, ry0 = INFINITY, rx1 = -INFINITY, ry1 = -INFINITY;
        double lx0 = INFINITY, ly0 = INFINITY, lx1 = -INFINITY, ly1 = -INFINITY;
        for (int c = 0; c < 3; ++c) {
            const double X = fp[2 * v[c]], Y = fp[2 * v[c] + 1];
            const double LX = G[0] + (double)dxy[2 * v[c]], LY = G[1] + (double)dxy[2 * v[c] + 1];
            rx0 = fmin(rx0, X); rx1 = fmax(rx1, X); ry0 = fmin(ry0, Y); ry1 = fmax(ry1, Y);
            lx0 = fmin(lx0, LX); lx1 = fmax(lx1, LX); ly0 = fmin(ly0, LY); ly1 = fmax(ly1, LY);
        }
        const double ext_r = fmax(rx1 - rx0, ry1 - ry0), ext_l = fmax(lx1 - lx0, ly1 - ly0);
        if (ext_r > OR_WARP_STRETCH * ext_l) continue;
        if (warp_edge(fp + 2 * v[0], fp + 2 * v[1], fp + 2 * v[2]) == 0.0) continue;
        keep[k] = 1;
        box[4 * k] = rx0; box[4 * k + 1] = ry0; box[4 * k + 2] = rx1; box[4 * k + 3] = ry1;
        gx0 = fmin(gx0, rx0); gy0 = fmin(gy0, ry0); gx1 = fmax(gx1, rx1); gy1 = fmax(gy1, ry1);
    }
    /* uniform bins over the kept boxes */
    const int NB = 1024;
    int64_t* cnt = (int64_t*)calloc((size_t)NB * NB + 1, sizeof(int64_t));
    const double bw = (gx1 - gx0) / NB, bh = (gy1 - gy0) / NB;
    const int have = gx0 < gx1 && gy0 < gy1;
#define OR_BIN_X(X) ((int)fmin(NB - 1.0, fmax(0.0, floor(((X) - gx0) / bw))))
#define OR_BIN_Y(Y) ((int)fmin(NB - 1.0, fmax(0.0, floor(((Y) - gy0) / bh))))
    if (have)
        for (int64_t k = 0; k < m; ++k) {
            if (!keep[k]) continue;
            for (int by = OR_BIN_Y(box[4 * k + 1]); by <= OR_BIN_Y(box[4 * k + 3]); ++by)
                for (int bx = OR_BIN_X(box[4 * k]); bx <= OR_BIN_X(box[4 * k + 2]); ++bx) cnt[by * NB + bx + 1]++;
        }
    for (int64_t b = 0; b < (int64_t)NB * NB; ++b) cnt[b + 1] += cnt[b];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)NB * NB);
    memcpy(fill, cnt, sizeof(int64_t) * (size_t)NB * NB);
    int64_t* items = (int64_t*)malloc(sizeof(int64_t) * (size_t)(cnt[(int64_t)NB * NB] + 1));
    if (have)
        for (int64_t k = 0; k < m; ++k) {
            if (!keep[k]) continue;
            for (int by = OR_BIN_Y(box[4 * k + 1]); by <= OR_BIN_Y(box[4 * k + 3]); ++by)
                for (int bx = OR_BIN_X(box[4 * k]); bx <= OR_BIN_X(box[4 * k + 2]); ++bx)
                    items[fill[by * NB + bx]++] = k;
        }
    /* coverage and the winner of every right texel */
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t c = 0; c < n; ++c) {
        tri_win[c] = -1;
        flag[c] = 0;
        if (!have) continue;
        const double Cp[2] = {G[0] + (double)dxy[2 * c], G[1] + (double)dxy[2 * c + 1]};
        if (Cp[0] < gx0 || Cp[0] > gx1 || Cp[1] < gy0 || Cp[1] > gy1) continue;
        const int64_t b = (int64_t)OR_BIN_Y(Cp[1]) * NB + OR_BIN_X(Cp[0]);
        uint64_t best = UINT64_MAX;
        int64_t best_k = -1;
        double best_b[3] = {0, 0, 0}, best_s = 0;
        for (int64_t q = cnt[b]; q < cnt[b + 1]; ++q) {
            const int64_t k = items[q];
            const int64_t* v = tv + 3 * k;
            const double* V0 = fp + 2 * v[0];
            const double* V1 = fp + 2 * v[1];
            const double* V2 = fp + 2 * v[2];
            const double A = warp_edge(V0, V1, V2);
            const double e0 = warp_edge(V1, V2, Cp), e1 = warp_edge(V2, V0, Cp), e2 = warp_edge(V0, V1, Cp);
            const int in = A > 0.0 ? (e0 >= 0.0 && e1 >= 0.0 && e2 >= 0.0) : (e0 <= 0.0 && e1 <= 0.0 && e2 <= 0.0);
            if (!in) continue;
            const double b0 = e0 / A, b1 = e1 / A, b2 = e2 / A;
            const double s = (b0 / (double)zr[v[0]] + b1 / (double)zr[v[1]]) + b2 / (double)zr[v[2]];
            const float depth = (float)(1.0 / s);
            uint32_t zb;
            memcpy(&zb, &depth, 4);
            const uint64_t key = ((uint64_t)zb << 32) | (uint64_t)(uint32_t)tid[k];
            if (key < best) {
                best = key;
                best_k = k;
                best_b[0] = b0; best_b[1] = b1; best_b[2] = b2;
                best_s = s;
            }
        }
        if (best_k < 0) continue;
        tri_win[c] = tid[best_k];
        if (depth_win) {
            const uint32_t zb = (uint32_t)(best >> 32);
            memcpy(&depth_win[c], &zb, 4);
        }
        const int64_t* v = tv + 3 * best_k;
        double w[3];
        for (int q = 0; q < 3; ++q) w[q] = (best_b[q] / (double)zr[v[q]]) / best_s;
        for (int ch = 0; ch < 4; ++ch)
            rgba_right[4 * c + ch] = (float)((w[0] * (double)rgba_left[4 * v[0] + ch] +
                                              w[1] * (double)rgba_left[4 * v[1] + ch]) +
                                             w[2] * (double)rgba_left[4 * v[2] + ch]);
        int top = 0;
        if (w[1] > w[top]) top = 1;
        if (w[2] > w[top]) top = 2;
        id_right[c] = hit_id[v[top]];
    }
    /* flags around triangles that use a flagged left texel */
    if (lflag && have)
        for (int64_t k = 0; k < m; ++k) {
            const int64_t* v = tv + 3 * k;
            if (!lflag[v[0]] && !lflag[v[1]] && !lflag[v[2]]) continue;
            double x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY, lw = 0.0;
            double lx0 = INFINITY, ly0 = INFINITY, lx1 = -INFINITY, ly1 = -INFINITY;
            for (int c = 0; c < 3; ++c) {
                const double LX = G[0] + (double)dxy[2 * v[c]], LY = G[1] + (double)dxy[2 * v[c] + 1];
                lx0 = fmin(lx0, LX); lx1 = fmax(lx1, LX); ly0 = fmin(ly0, LY); ly1 = fmax(ly1, LY);
                if (!ok[v[c]]) continue;
                x0 = fmin(x0, fp[2 * v[c]]); x1 = fmax(x1, fp[2 * v[c]]);
                y0 = fmin(y0, fp[2 * v[c] + 1]); y1 = fmax(y1, fp[2 * v[c] + 1]);
            }
            if (!(x0 <= x1)) continue;
            lw = fmax(lx1 - lx0, ly1 - ly0);
            const double wx = fmax(x1 - x0, lw), wy = fmax(y1 - y0, lw);
            x0 -= wx; x1 += wx; y0 -= wy; y1 += wy;
            for (int64_t c = 0; c < n; ++c) {
                const double X = G[0] + (double)dxy[2 * c], Y = G[1] + (double)dxy[2 * c + 1];
                if (X >= x0 && X <= x1 && Y >= y0 && Y <= y1) flag[c] = 1;
            }
        }
#undef OR_BIN_X
#undef OR_BIN_Y
    free(items);
    free(fill);
    free(cnt);
    free(box);
    free(keep);
    free(tid);
    free(tv);
    free(ok);
    free(zr);
    free(fp);
}
