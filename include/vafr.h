/*
 * vafr.h -- C ABI of the MI355X-native VaFR hot path.
 *
 * Visual-acuity-consistent foveated rendering ("Visual Acuity Consistent
 * Foveated Rendering towards Retinal Resolution", Zhang, Gai, Li, arXiv
 * 2503.23410): a constant-size log-polar (LP) buffer whose radial axis and
 * shading rate follow the acuity model (Sec. 3.2, 3.3) is shaded with one
 * ray-cast sample per texel (Sec. 6.1) and inverse-mapped onto every display
 * pixel (Sec. 3.2.3).  The LMFR and LaFR log-polar mappings (Sec. 3.1
 * Eq. (1), Sec. 4.1 Eq. (14), Eq. (15)) and a full-resolution ray cast are
 * the same-GPU comparisons.
 *
 * Conventions
 *  - Every call returns int: VAFR_OK (0) or a negative VAFR_E_* code; the
 *    message of the last failure on the calling thread is vafr_last_error().
 *    No C++ exception crosses the ABI.
 *  - Handles (vafr_layout, vafr_scene) are owned by the library, immutable
 *    after creation and safe to share across threads and streams; free them
 *    with the matching *_destroy.
 *  - Buffer arguments named *_dev are device pointers owned by the caller
 *    (e.g. from torch tensors) on the device that is current at the call.
 *    Host arrays are read during the call only.
 *  - Per-frame calls are asynchronous on the caller's stream.  Only
 *    vafr_scene_create and the first use of a layout on a device (table
 *    upload) synchronise.
 *  - Angles are in degrees.  Display pixel coordinates are continuous:
 *    pixel (x, y) covers [x, x+1) x [y, y+1), x grows right, y grows down.
 *  - Colours are linear FP32 RGBA (alpha = 1), no tone map.
 */
#ifndef VAFR_H
#define VAFR_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VAFR_OK 0
#define VAFR_E_ARG (-1)          /* invalid argument (checked before any launch) */
#define VAFR_E_OOM (-2)          /* host or device allocation failed            */
#define VAFR_E_HIP (-3)          /* a HIP runtime call failed / no device       */
#define VAFR_E_UNSUPPORTED (-4)  /* valid request the library cannot serve      */
#define VAFR_E_BUDGET (-5)       /* request exceeds a memory budget             */
#define VAFR_E_LATE (-6)         /* request dropped: it could not complete by its
                                    deadline, or a newer request replaced it   */
#define VAFR_E_TIMEOUT (-7)      /* the device made no progress within a
                                    watchdog limit; the work was abandoned     */

/* Message of the last failure on this thread ("" if none).  The pointer
 * stays valid until the next failing call on the same thread. */
const char* vafr_last_error(void);

/* ABI version: bumped on any incompatible change of this header. */
int vafr_abi_version(void);

/* ------------------------------------------------------------------ types */

/* Display: resolution and full field of view (Sec. 3.2.1, Eq. (3) relates
 * pixels to eccentricity through the film-plane pitch). */
typedef struct {
    int32_t width, height;
    double fov_x_deg, fov_y_deg;   /* in (0, 180) */
} vafr_display;

/* Acuity pivots (Sec. 3.3): MAR 1/cpd is linear between consecutive
 * (ecc_deg[k], cpd[k]); ecc_deg[0] must be 0 and strictly increasing;
 * cpd > 0; 2 <= n_pivots <= 16; 0 < e_max_deg < 90.  Passing NULL for the
 * acuity selects the paper's pivots {0,10,20,30,60} deg -> {40,10,6,5,4} cpd
 * and e_max = 60 deg (Sec. 3.2.2), isotropic.
 *
 * Anisotropy (Sec. 9, Eq. (19)): the tangential shading rate is Delta(e)
 * times the radial one, so column i gets ceil(Delta(e_i) l(e_i)) rows.
 * Delta is linear between (aniso_ecc_deg[k], aniso_delta[k]) and constant
 * before the first and after the last point; 0 <= n_aniso <= 16 (0: Delta =
 * 1), eccentricities strictly increasing, 0 < delta <= 16. */
typedef struct {
    int32_t n_pivots;
    const double* ecc_deg;
    const double* cpd;
    double e_max_deg;
    int32_t n_aniso;
    const double* aniso_ecc_deg;
    const double* aniso_delta;
} vafr_acuity;

/* Device-adapted curve (Sec. 3.3): pivots of f_cap(e) = min(f(e), cap_cpd)
 * for the pivot curve `in` (NULL: the paper's pivots).  The MAR of f_cap is
 * max(1/f, 1/cap): each original pivot keeps its eccentricity with
 * min(cpd, cap), and a pivot is inserted where a segment's MAR crosses
 * 1/cap.  Writes *n_out <= max_out pivots to ecc_out / cpd_out (e_max and
 * anisotropy of `in` are not copied).  Errors: VAFR_E_ARG for an invalid
 * curve, cap <= 0 or max_out too small. */
int vafr_acuity_capped(const vafr_acuity* in, double cap_cpd, double* ecc_out, double* cpd_out, int32_t max_out,
                       int32_t* n_out);

/* Pinhole camera: eye position and an orthonormal basis; the film plane is
 * at unit distance along forward, film y points along -up. */
typedef struct {
    float eye[3], right[3], up[3], forward[3];
} vafr_camera;

/* Gaze point in continuous display-pixel coordinates (may lie off screen). */
typedef struct {
    double x_px, y_px;
} vafr_gaze;

#define VAFR_SHADE_LAMBERT 0
#define VAFR_SHADE_PATH 1

/* Shading.  Lambert mode: miss -> background; hit -> albedo(id) *
 * (ambient + light_rgb * max(0, n.l) * vis), one shadow ray when
 * shadow_rays = 1.  Path mode: one sample, next-event estimation to the
 * directional light at each vertex and `bounces` cosine-weighted
 * continuation rays; random numbers are keyed by (seed, frame, view, texel).
 * light_dir points toward the light: any finite non-zero vector, which the
 * library normalises (FP64 from the FP32 components, squares summed as
 * (x x + y y) + z z, each component divided by the square root and rounded
 * once to FP32); VAFR_E_ARG for a zero or non-finite vector. */
typedef struct {
    float light_dir[3];
    float light_rgb[3];
    float ambient[3];
    float background[3];
    int32_t shadow_rays;   /* 0 or 1 */
    int32_t mode;          /* VAFR_SHADE_LAMBERT or VAFR_SHADE_PATH */
    int32_t bounces;       /* path mode: 0..8 */
    uint32_t frame;        /* path mode key */
    uint32_t view;         /* path mode key */
    uint32_t pad_;
    uint64_t seed;         /* path mode key */
} vafr_shading;

#define VAFR_LAYOUT_VAFR 0
#define VAFR_LAYOUT_LMFR 1
#define VAFR_LAYOUT_LAFR 2

/* Layout dimensions.  VaFR: n_cols columns of n_rows[i] texels stored
 * column-major and packed (texel k of column i is col_off[i] + j);
 * LMFR / LaFR: a dense n_cols x max_rows buffer, k = i * max_rows + j. */
typedef struct {
    int32_t kind;          /* VAFR_LAYOUT_VAFR, VAFR_LAYOUT_LMFR or VAFR_LAYOUT_LAFR */
    int32_t n_cols;
    int32_t max_rows;
    int32_t width, height; /* display the layout was made for */
    int64_t n_texels;
} vafr_dims;

typedef struct vafr_layout_s* vafr_layout;
typedef struct vafr_scene_s* vafr_scene;

/* ----------------------------------------------------------------- layout */

/* VaFR LP layout (Sec. 3.2.1-3.2.3, Sec. 3.3 Eq. (12)): FP64 segment
 * constants of u(e) (Eq. (5)), ceil(u(e_max)) columns sampled at their
 * centres, n_i = ceil(l(e_i)) rows (Eq. (9); ceil(Delta(e_i) l(e_i)) with
 * anisotropy, Eq. (19)) at polar angles
 * 360 (j + 1/2)/n_i, and per texel the FP32 film-plane offset
 * tan(e_i) (cos, sin) of its screen point from the gaze point.  The tables do
 * not depend on the display; the display fixes the pixel pitch used by
 * vafr_shade_lp / vafr_reconstruct.  Host-only; tables are uploaded to a
 * device on first use there.  Errors: VAFR_E_ARG for an invalid display or
 * acuity, VAFR_E_OOM. */
int vafr_lp_layout(const vafr_display* display, const vafr_acuity* acuity, vafr_layout* out);

/* LMFR comparison layout (Sec. 3.1 Eq. (1), Sec. 4.1 Eq. (14), Sec. 5.2):
 * round(W/delta) x round(H/delta) texels, kernel K(z) = z^alpha.
 * delta >= 1, alpha > 0. */
int lmfr_lp_layout(const vafr_display* display, double delta, double alpha, vafr_layout* out);

/* LaFR comparison layout (Sec. 4.1 Eq. (15), Sec. 4.5, Sec. 5.2): the same
 * round(W/delta) x round(H/delta) buffer as LMFR, with the two-piece LaFR
 * kernel.  Columns at u/w <= U_ef hold z = (u/w)^Fa / (1 - Fa) (eccentricity
 * up to 4.89 deg); the rest follow the arccos piece with exponent beta/0.7,
 * reaching z = 1 at the last column edge.  Per gaze, with ln L as for LMFR
 * and c_r the film pitch of one pixel:
 *   Z_ef = ln(tan 4.89 deg / c_r) / ln L,
 *   Fa   = 1 - log_{Z_ef}((alpha Z_ef)^(1 - a) / (1 - a)),
 *   U_ef = (Z_ef (1 - Fa))^(1 / Fa).
 * a is LMFR's kernel exponent in the buffer-to-screen direction (1/4 for
 * LMFR's z^4); LaFR's own parameters are alpha = 0.85, beta = 0.7.
 * delta >= 1, 0 < a < 1, 0 < alpha <= 1, 0 < beta <= 16.  The shading and
 * reconstruction calls fail with VAFR_E_ARG for a gaze at which Z_ef or Fa
 * leaves (0, 1). */
int lafr_lp_layout(const vafr_display* display, double delta, double a, double alpha, double beta,
                   vafr_layout* out);

int vafr_layout_dims(vafr_layout layout, vafr_dims* out);

/* Host views of the layout tables (valid until vafr_layout_destroy):
 * n_rows[n_cols], col_off[n_cols + 1], texel_dxy[2 * n_texels] (VaFR only;
 * NULL for LMFR / LaFR).  These are the bit-exact contract of the layout. */
int vafr_layout_tables(vafr_layout layout, const int32_t** n_rows, const int64_t** col_off,
                       const float** texel_dxy);

void vafr_layout_destroy(vafr_layout layout);

/* ------------------------------------------------------------------ scene */

/* Triangle scene: xyz[3 * n_verts] FP32 positions, tri[3 * n_tris] vertex
 * indices; triangle ids are positions in tri[].  Builds a binned-SAH BVH on
 * the host and, when a HIP device is present, uploads it to the current
 * device (synchronous).  0 <= n_tris < 2^27.  Errors: VAFR_E_ARG for an
 * index out of range or a non-finite vertex, VAFR_E_OOM, VAFR_E_HIP. */
int vafr_scene_create(const float* xyz, int64_t n_verts, const int32_t* tri, int64_t n_tris, vafr_scene* out);

typedef struct {
    int64_t n_tris;
    int64_t n_nodes;       /* internal (4-wide) nodes */
    int64_t n_leaves;
    int32_t max_depth;     /* levels of the binary build tree below the root */
    int32_t on_device;     /* 1 if uploaded */
    int64_t device_bytes;
    double build_ms;
    int32_t stack_entries; /* traversal stack entries per ray in LDS (more spill to scratch) */
    int32_t max_stack;     /* most entries a traversal can hold */
} vafr_scene_info;

int vafr_scene_get_info(vafr_scene scene, vafr_scene_info* out);

/* Host copies of the BVH for structural checks: nodes[16 * n_nodes] as
 * stored on the device (per node: origin x, y, z, scale z; 8-bit plane
 * codes of four child boxes, x-lo, x-hi, y-lo, y-hi, z-lo, z-hi, child c in
 * byte c, then scale x, scale y (FP32 powers of two); four child references,
 * INT32_MIN for an empty slot) and
 * tri_order[n_tris] (original id of each stored triangle).  Either may be
 * NULL. */
int vafr_scene_export(vafr_scene scene, float* nodes, int32_t* tri_order);

void vafr_scene_destroy(vafr_scene scene);

/* ---------------------------------------------------------- per-frame work */

/* Shade an LP buffer (Sec. 6.1): one ray per texel from the eye through
 * the texel's screen point (gaze + offset), closest hit over the scene BVH
 * with the FP32 watertight test (ties broken by the smaller triangle id),
 * then the shading model.  lp_rgba_dev[4 * n_texels]; hit_id_dev[n_texels]
 * (nullable) receives the primary hit triangle id or -1.  Works with a VaFR
 * layout; lmfr_shade_lp and lafr_shade_lp are the same call for an LMFR and
 * a LaFR layout. */
int vafr_shade_lp(vafr_scene scene, const vafr_camera* cam, vafr_gaze gaze, const vafr_shading* shading,
                  vafr_layout layout, float* lp_rgba_dev, int32_t* hit_id_dev, hipStream_t stream);

int lmfr_shade_lp(vafr_scene scene, const vafr_camera* cam, vafr_gaze gaze, const vafr_shading* shading,
                  vafr_layout layout, float* lp_rgba_dev, int32_t* hit_id_dev, hipStream_t stream);

int lafr_shade_lp(vafr_scene scene, const vafr_camera* cam, vafr_gaze gaze, const vafr_shading* shading,
                  vafr_layout layout, float* lp_rgba_dev, int32_t* hit_id_dev, hipStream_t stream);

/* Anti-aliasing inside the LP buffer (Sec. 3.4: FXAA on the LP buffer before
 * the inverse map).  FXAA's steps (Lottes 2009) on the polar grid: along the
 * angle a texel's neighbours are the adjacent rows of its column (cyclic),
 * along the radius the inner and outer columns sampled at its angle (linear
 * in rows; columns clamp at the ends).  A texel whose luma range over itself
 * and its four neighbours is below max(1/16, 1/8 of the largest luma) is
 * copied; otherwise the edge normal follows the larger luma curvature, the
 * ends of the edge are searched at offsets 1, 2, 3, 4, 6, 8 along it, and the
 * texel is blended toward the neighbour across the edge by
 * max(edge term, 0.75 x sub-texel term).  lp_in_dev and lp_out_dev hold
 * 4 * n_texels floats of a VaFR layout and must not overlap.  Errors:
 * VAFR_E_ARG (NULL or overlapping buffers), VAFR_E_UNSUPPORTED (LMFR
 * layout), VAFR_E_HIP. */
int vafr_fxaa_lp(vafr_layout layout, const float* lp_in_dev, float* lp_out_dev, hipStream_t stream);

/* Binocular reprojection (Sec. 5.1, VaFR_Rep): shades the left eye's LP
 * buffer as vafr_shade_lp does, then builds the right eye's from it by
 * forward grid warping.  The left texels' primary hit points p = fma(t, d,
 * o) form a mesh in LP topology: the band between columns s and s + 1 is
 * triangulated by a zipper over the two columns' texels merged by angle.
 * Every vertex is projected onto the right film plane (FP32: q = p - eye;
 * x, y, z = dot(q, right / up / forward) summed left to right; film point
 * (x / z, -(y / z))); a triangle is dropped when a vertex missed, lies
 * behind the right eye or projects to a non-finite point, when its depths
 * differ by more than 1/10, when it is stretched to more than twice its
 * left film size, or when its area is zero.  A right texel whose sample
 * point (gaze + film offset) lies inside a kept triangle (FP64 edge
 * functions) takes the triangle's perspective-correct depth; the least
 * (depth, triangle id) wins the texel, whose colour is the
 * perspective-correct interpolation of the three left colours and whose hit
 * id is that of the vertex of largest weight.  Texels no kept triangle
 * covers are ray-cast with the right camera (only those: they are listed
 * and traced as one compacted launch).  Both eyes use the gaze display
 * point.
 * workspace_dev: caller-owned device memory of vafr_rep_workspace_bytes()
 * bytes (hit points, texel keys, list of uncovered texels), 16-byte
 * aligned, reused across calls on one stream (calls that overlap on one
 * workspace race).  hit_left / hit_right are nullable.  The LP buffers,
 * hit-id buffers and workspace must not overlap.  right_stream (nullable or
 * equal to stream: one stream) receives the ray casting of the uncovered
 * texels, ordered after the warp on stream; lp_right / hit_right are then
 * complete in right_stream's order, lp_left / hit_left in stream's, and the
 * workspace stays in use until right_stream's work is done.  A caller can
 * so overlap that latency-bound pass with work on stream, such as the left
 * eye's inverse map.  Errors: VAFR_E_ARG (NULL, overlapping or misaligned
 * buffers, small workspace, invalid camera / shading / gaze),
 * VAFR_E_UNSUPPORTED (LMFR / LaFR layout), VAFR_E_HIP. */
int vafr_rep_workspace_bytes(vafr_layout layout, int64_t* bytes);
int vafr_shade_lp_rep(vafr_scene scene, const vafr_camera* cam_left, const vafr_camera* cam_right, vafr_gaze gaze,
                      const vafr_shading* shading, vafr_layout layout, float* lp_left_dev, float* lp_right_dev,
                      int32_t* hit_left_dev, int32_t* hit_right_dev, void* workspace_dev, int64_t workspace_bytes,
                      hipStream_t stream, hipStream_t right_stream);

/* Allocation-free reprojection, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): vafr_shade_lp_rep on one stream, with its workspace
 * in a static device array of 32 MiB per GPU (held until the process ends)
 * instead of caller memory; the call allocates nothing.  Layouts of up to
 * 1,198,372 texels (vafr_rep_workspace_bytes <= 32 MiB; the paper's acuity
 * layout has 1,063,314): larger ones fail with VAFR_E_BUDGET before any
 * launch.  The layout's tables must already be on the current device (any
 * per-frame call with the layout uploads them), else VAFR_E_UNSUPPORTED.
 * Every call on one GPU shares that GPU's array, which keeps the last
 * call's contents (the kernels clear what must start at zero): calls that
 * overlap on one GPU, on any streams, race.  Buffers and other errors as
 * vafr_shade_lp_rep. */
int vafr_shade_lp_rep_noalloc(vafr_scene scene, const vafr_camera* cam_left, const vafr_camera* cam_right,
                              vafr_gaze gaze, const vafr_shading* shading, vafr_layout layout, float* lp_left_dev,
                              float* lp_right_dev, int32_t* hit_left_dev, int32_t* hit_right_dev, hipStream_t stream);

/* Inverse map (Sec. 3.2.3, Eqs. (10)-(11)): every display pixel centre is
 * mapped to (u, theta) and the LP buffer is sampled with a two-column,
 * angle-consistent bilinear filter (u clamped to the first/last column
 * centre, theta wrapping).  img_rgba_dev[4 * W * H], row-major. */
int vafr_reconstruct(vafr_layout layout, vafr_gaze gaze, const float* lp_rgba_dev, float* img_rgba_dev,
                     hipStream_t stream);

/* LMFR inverse map: Eq. (1) with K(z) = z^alpha, bilinear, u clamped,
 * v wrapping. */
int lmfr_reconstruct(vafr_layout layout, vafr_gaze gaze, const float* lp_rgba_dev, float* img_rgba_dev,
                     hipStream_t stream);

/* LaFR inverse map: Eq. (15) forward (pixel radius clamped to >= 1 pixel),
 * then the same bilinear sampling as lmfr_reconstruct. */
int lafr_reconstruct(vafr_layout layout, vafr_gaze gaze, const float* lp_rgba_dev, float* img_rgba_dev,
                     hipStream_t stream);

/* Full-resolution ray cast (Sec. 5.2 "GT"): one ray per display pixel
 * centre, shaded as vafr_shade_lp, written to img_rgba_dev[4 * W * H];
 * hit_id_dev[W * H] nullable. */
int full_shade(vafr_scene scene, const vafr_camera* cam, const vafr_display* display, const vafr_shading* shading,
               float* img_rgba_dev, int32_t* hit_id_dev, hipStream_t stream);

/* ---------------------------------------------------------------- batches */

#define VAFR_VIEW_VAFR 0
#define VAFR_VIEW_LMFR 1
#define VAFR_VIEW_FULL 2
#define VAFR_VIEW_LAFR 3

/* One view of a batched frame.  VAFR / LMFR / LAFR views shade layout's LP buffer
 * into lp_rgba_dev and, when img_rgba_dev is not NULL, inverse-map it onto
 * the layout's display; FULL views ray-cast every pixel of `display` into
 * img_rgba_dev.  Same buffer contracts as the per-view calls. */
typedef struct {
    int32_t kind;            /* VAFR_VIEW_* */
    int32_t pad_;
    vafr_scene scene;
    vafr_layout layout;      /* VAFR / LMFR / LAFR views; NULL for FULL */
    vafr_display display;    /* FULL views only */
    vafr_camera camera;
    vafr_gaze gaze;
    vafr_shading shading;
    float* lp_rgba_dev;      /* VAFR / LMFR / LAFR views */
    int32_t* hit_id_dev;     /* nullable */
    float* img_rgba_dev;     /* nullable for LP-only VAFR / LMFR / LAFR views */
} vafr_view;

/* Launch shape of a batch: traversal workgroup size (64, 128 or 256 rays),
 * display rows each reconstruction thread writes (1, 2, 4 or 8; a
 * workgroup of 256 threads covers 64 x 4 recon_rows pixels) and whether
 * frames are replayed from a hipGraph. */
typedef struct {
    int32_t trace_block;
    int32_t recon_rows;
    int32_t use_graph;
} vafr_batch_config;

typedef struct vafr_batch_s* vafr_batch;

/* A batch runner for up to max_views views per frame (1..256).  It owns
 * pinned host and device descriptor tables (a ring of 4 frames in flight).
 * cfg may be NULL for the defaults {128, 4, 1}. */
int vafr_batch_create(int32_t max_views, const vafr_batch_config* cfg, vafr_batch* out);

/* One frame of n_views views on `stream`: ONE traversal launch covering the
 * rays of every view (workgroups are assigned to views by a running count)
 * and ONE reconstruction launch covering every display of the VaFR / LMFR
 * views.  Two VaFR views with the same layout, gaze and display (the eyes of
 * a binocular frame) share their reconstruction workgroups: each pixel's
 * texel positions and weights are found once and applied to both LP
 * buffers.  Path-mode views run in phases: bounces 0 and 1 in the traversal
 * launch, and each bounce b >= 2 in a launch of its own over the paths still
 * alive, one per thread; between launches each path's state (next ray,
 * throughput, radiance) lives in memory the batch allocates, 72 bytes per
 * ray of those views, per descriptor slot on first use.  With
 * use_graph the sequence (descriptor upload, kernels) is a hipGraph built
 * once per launch shape; later frames only update the node parameters and
 * replay it.  Results are identical to the per-view calls.  Blocks the host
 * only when all 4 descriptor slots are still in flight. */
int vafr_batch_run(vafr_batch batch, const vafr_view* views, int32_t n_views, hipStream_t stream);

/* Times every traversal workgroup size and reconstruction tile height on
 * these views (reps frames each, on `stream`) and keeps the fastest in the
 * batch's configuration; the choice is also returned in *chosen (nullable). */
int vafr_batch_autotune(vafr_batch batch, const vafr_view* views, int32_t n_views, int32_t reps, hipStream_t stream,
                        vafr_batch_config* chosen);

int vafr_batch_get_config(vafr_batch batch, vafr_batch_config* out);
int vafr_batch_set_config(vafr_batch batch, const vafr_batch_config* cfg);

/* Stage timing: with profiling on, every frame records events around its
 * descriptor upload, traversal launch and reconstruction launch (event-record
 * nodes in graph mode); durations are read when a slot is reused, so timing
 * adds no host synchronisation.  vafr_batch_stage_ms waits for the frames in
 * flight and returns the mean (upload, traversal, reconstruction) durations
 * in ms over all frames run since profiling was switched on (count in
 * *frames, nullable).  vafr_batch_set_profiling resets the accumulators. */
int vafr_batch_set_profiling(vafr_batch batch, int32_t on);
int vafr_batch_stage_ms(vafr_batch batch, float* mean3, int64_t* frames);

/* Waits for the batch's frames in flight and frees it. */
void vafr_batch_destroy(vafr_batch batch);

/* ---------------------------------------------------------------- serving */

typedef struct vafr_server_s* vafr_server;

typedef struct {
    int32_t max_views_per_launch;  /* views per batched launch (2 per request), 2..256 */
    int32_t max_inflight;          /* launches on the device at once, 1..64 (<= 4 per stream avoids
                                      host waits on descriptor slots) */
    int32_t n_streams;             /* streams the launches are spread over, 1..8 */
    int32_t max_queue;             /* waiting requests beyond which submissions are refused */
    int64_t hbm_budget_bytes;      /* bound on per-request buffers (LP buffers + display images) */
    vafr_batch_config batch;       /* launch shape of every batch; use_graph = 0 suits serving (each new
                                      mix of requests would be a new graph to instantiate on the
                                      dispatcher thread, for little replay gain on multi-ms launches) */
    int32_t simulate;              /* 1: no GPU; a launch of R Mrays (LP texels) and P Mpixels finishes
                                      sim_ms_per_launch + R sim_ms_per_mray + P sim_ms_per_mpix after the
                                      simulated device is free (capacity planning and policy tests) */
    int32_t pad_;
    double sim_ms_per_launch, sim_ms_per_mray, sim_ms_per_mpix;
    double frame_budget_ms;        /* > 0: a request must complete within this many ms of its submission
                                      (or within its own deadline_ms if that is smaller); 0 = none */
    int32_t latest_only;           /* 1: a new request of a headset replaces that headset's requests
                                      not yet launched (they finish with VAFR_E_LATE) */
    int32_t pad2_;
    double watchdog_ms;            /* > 0: stall limit.  When launches are in flight and none has
                                      completed for this many ms, the server gives them up (see
                                      vafr_server_create); 0 = no watchdog */
} vafr_server_config;

/* A headset: resident scene and VaFR layout (display), one camera per eye
 * and its shading (frame / view keys are set per request: frame from the
 * request, view = 2 * headset + eye). */
typedef struct {
    vafr_scene scene;
    vafr_layout layout;
    vafr_camera camera[2];
    vafr_shading shading;
} vafr_headset;

/* One binocular frame request: both eyes use the gaze display point. */
typedef struct {
    int32_t headset;
    uint32_t frame;
    vafr_gaze gaze;
    double deadline_ms;            /* latest completion, ms after submit; 0 = none (frame_budget_ms of
                                      the server applies if set) */
    uint64_t user_tag;
} vafr_request;

/* A finished request.  status VAFR_OK: the images (and LP buffers) of both
 * eyes are ready at the device pointers, which stay valid until
 * vafr_server_release(slot).  VAFR_E_LATE: dropped before launch because it
 * could not complete by its deadline, or replaced by a newer request of the
 * headset.  VAFR_E_BUDGET: dropped while draining without memory.
 * VAFR_E_TIMEOUT: launched (or waiting) when the watchdog gave up on the
 * device.  No slot and nothing to release for any error status.  Times are
 * ms on the server's clock. */
typedef struct {
    uint64_t user_tag;
    int32_t headset;
    uint32_t frame;
    int32_t status;
    int32_t slot;
    double submit_ms, launch_ms, done_ms;
    const float* img_rgba_dev[2];
    const float* lp_rgba_dev[2];
} vafr_result;

/* dropped counts every request finished with an error status; late and
 * superseded count the VAFR_E_LATE drops by cause, stalled the
 * VAFR_E_TIMEOUT ones. */
typedef struct {
    int64_t submitted, completed, refused, deferred, dropped, launches, views_launched, bytes_in_use;
    int32_t waiting, inflight;
    int64_t late, superseded, stalled;
} vafr_server_stats;

/* Starts the dispatcher thread on the current device.  Requests are
 * admitted in arrival order when a buffer set fits the budget (deferred
 * otherwise); every free launch slot takes all admitted requests at the
 * head of the queue (up to max_views_per_launch / 2) into one batched frame
 * (vafr_batch_run) on the least busy stream, so requests that arrive while
 * others run join the next launch.  Results equal those of the request
 * rendered alone (kernels are per view and deterministic).
 *
 * Requests with a deadline go through a device-time model: a per-launch
 * cost plus a cost per request of each headset, seeded from the headset's
 * ray and pixel counts and corrected after every launch by its measured
 * device time.  A launch takes requests from the queue head while the
 * predicted end of the device's queued work plus the launch meets every
 * included deadline; a request that cannot meet its deadline even in a
 * launch of its own is dropped (VAFR_E_LATE).
 *
 * Watchdog (watchdog_ms > 0): the device is taken to have stalled when work
 * is in flight and no launch has completed for watchdog_ms (measured from
 * the last completion, or from the launch that found the device idle, so a
 * deep but moving queue never trips it).  The server then finishes every
 * launched and waiting request with VAFR_E_TIMEOUT, keeps the buffers of the
 * abandoned launches out of the pool (the device may still write them),
 * refuses further submissions with VAFR_E_TIMEOUT, and vafr_server_destroy
 * neither waits for nor frees device objects that abandoned work may still
 * use (they are leaked if that work has not finished by then). */
int vafr_server_create(const vafr_server_config* cfg, vafr_server* out);
int vafr_server_add_headset(vafr_server server, const vafr_headset* headset, int32_t* id);
/* Non-blocking; VAFR_E_BUDGET when the queue is full (counted as refused),
 * VAFR_E_TIMEOUT after a watchdog stall. */
int vafr_server_submit(vafr_server server, const vafr_request* request);
/* Up to max finished requests, oldest first; *n_out set to the count.
 * Returns VAFR_OK while it delivers results; once none is left it returns
 * the server's sticky error, if any (a failed launch: VAFR_E_HIP; a stall:
 * VAFR_E_TIMEOUT), so per-request statuses are always delivered first. */
int vafr_server_poll(vafr_server server, vafr_result* out, int32_t max, int32_t* n_out);
int vafr_server_release(vafr_server server, int32_t slot);
/* Waits until nothing is queued or in flight (VAFR_E_BUDGET on timeout). */
int vafr_server_wait_idle(vafr_server server, int32_t timeout_ms);
int vafr_server_get_stats(vafr_server server, vafr_server_stats* out);
/* Finishes in-flight work, drops requests that cannot be admitted, frees
 * every buffer (results not yet released become invalid). */
void vafr_server_destroy(vafr_server server);

/* ------------------------------------------------------------ diagnostics */

/* Work counting for roofline reports: traces exactly the rays that
 * vafr_shade_lp / lmfr_shade_lp would trace for this layout (kind taken from
 * the layout) and atomically adds to counters_dev[4] (device, caller-zeroed
 * unsigned 64-bit): primary rays, shadow rays, BVH node visits (each a test
 * of a node's four child boxes) and ray/triangle tests.  Writes no image. */
int vafr_count_work(vafr_scene scene, const vafr_camera* cam, vafr_gaze gaze, const vafr_shading* shading,
                    vafr_layout layout, unsigned long long* counters_dev, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* VAFR_H */
