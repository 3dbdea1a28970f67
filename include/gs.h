/* gs.h — C ABI of the gfx950 differentiable Gaussian-splatting rasterizer.
 *
 * The library renders a map of anisotropic 3D Gaussians from a pinhole camera and
 * differentiates the result with respect to every Gaussian parameter and the camera pose.
 * It follows Sec. "3D Gaussian Splatting Representation" of Gaussian-LIC2 (projection,
 * EWA covariance, eq:alpha, front-to-back compositing of eq:rendered_rgb, eq:rendered_depth
 * and eq:rendered_opacity, SH colour, eq:3dgs_jacobi for the pose), the fast tile-based cull
 * of Sec. "CUDA-Related Acceleration Strategies", and the sparse-LiDAR depth term of
 * eq:depth_loss.
 *
 * Conventions shared by every call:
 *   - All array pointers are DEVICE pointers, float32 unless stated. "[k][n]" is a set of k
 *     planes of n elements (SoA): component j of element i is at ptr[j*n + i].
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null stream) and
 *     returns GS_OK or an error code. Argument errors are detected on the host before any
 *     launch. No call allocates device memory except gs_batch_plan_create and
 *     gs_track_plan_create.
 *   - Buffers are owned by the caller and must stay valid until the stream work completes.
 *   - Gradient outputs are ACCUMULATED (+=): zero them before the first call.
 *   - Pixel centres sit at integer coordinates. A camera carries a render window
 *     (x0, y0, w, h) inside its full image; every image plane is window-sized, row-major.
 *   - Invalid Gaussians are not errors: a non-finite value, |q| = 0, a scale <= 0, a depth
 *     <= 0.2, an opacity < 1/255 or a footprint outside the window drops the Gaussian
 *     (zero tiles, zero gradient).
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *gs_stream_t; /* hipStream_t */

enum {
  GS_OK = 0,
  GS_ERR_INVALID_ARG = 1, /* null pointer, bad size, bad tile size, window outside the image ... */
  GS_ERR_HIP = 2,         /* a HIP launch or API call failed; see gs_last_error() */
  GS_ERR_UNSUPPORTED = 3, /* device is not gfx950, or a mode the plan was not made for */
  GS_ERR_CAPACITY = 4     /* reserved for host-side capacity checks (see gs_bins) */
};

enum { GS_MAX_VIEWS = 16 };
enum { GS_FWD = 1u, GS_BWD = 2u, GS_GRAPH = 4u };

/* Pinhole camera with world-to-camera pose (^C_W R, ^C p_W), Sec. "3D Gaussian Splatting
 * Representation". Host struct, passed by pointer. */
typedef struct gs_camera {
  int32_t width, height;  /* full image in pixels */
  int32_t x0, y0, w, h;   /* render window; 0 <= x0, x0 + w <= width, same for y */
  float fx, fy, cx, cy;   /* pixel = (fx x/z + cx, fy y/z + cy) */
  float R_cw[9];          /* row-major rotation world -> camera */
  float t_cw[3];          /* translation world -> camera */
  float bg[3];            /* background colour added as T_final * bg */
} gs_camera;

/* The Gaussian map (Sec. "3D Gaussian Splatting Representation"): mean [3][n]; linear scale
 * [3][n] (> 0); rotation quaternion [4][n] as (w, x, y, z), normalised inside the kernels;
 * opacity [n] in (0, 1); SH DC coefficients sh_dc [3][n] and higher-order coefficients
 * sh_rest [3*((deg+1)^2-1)][n] with plane 3*(k-1)+channel for basis k >= 1, kept apart from
 * the DC plane ("separated SH", Sec. "CUDA-Related Acceleration Strategies" b). sh_rest may
 * be NULL at degree 0. */
typedef struct gs_gaussians {
  int64_t n;
  int32_t sh_degree; /* 0..3 */
  const float *mean, *scale, *rot, *opacity, *sh_dc, *sh_rest;
} gs_gaussians;

/* Per-Gaussian splat records written by gs_preprocess (n = number of Gaussians x views).
 * card [n][16] (64 B per record, 64-B aligned, so that every later gather of a record
 * touches one memory line):
 *   words 0-3   (u, v, o, d): projected centre mu', opacity, camera-frame depth;
 *   words 4-7   (a, b, c, kappa^2): conic Sigma'^-1 = [[a, b], [b, c]] and the squared
 *               footprint radius 2 ln(255 o);
 *   words 8-11  (r, g, b, m): view-dependent colour max(0, SH . Y(dir) + 0.5); the bits of m
 *               (a float holding an integer bit pattern) mark the channels not clamped;
 *   words 12-13 int16 inclusive tile rectangle (tx0, ty0, tx1, ty1), -1 when n_tiles = 0;
 *   word 14     number of tiles kept (copy of n_tiles below);
 *   word 15     for rectangles of at most 32 tiles, bit t set when the t-th tile of the
 *               rectangle (row-major) passed the cull; 0 for larger rectangles.
 * n_tiles [n]  number of tiles kept after the alpha-max cull;
 * dkey    [n]  sort key: IEEE bits of d, or 0xFFFFFFFF when n_tiles = 0;
 * pose         optional (NULL: the camera's): device float [16], the world-to-camera pose
 *              R_cw (9, row-major), t_cw (3) and camera centre -R^T t (3) (+1 unused), read
 *              on the device by gs_preprocess and gs_render_bwd in place of cam->R_cw / t_cw,
 *              so a pose computed on the device (gs_pose_left_update) needs no host round
 *              trip. Single-view calls only. */
typedef struct gs_projected {
  float *card;
  uint32_t *n_tiles;
  uint32_t *dkey;
  const float *pose;
} gs_projected;

/* Tile lists (Sec. "CUDA-Related Acceleration Strategies", fast tile-based culling; depth
 * order of eq:rendered_rgb). Tiles are tile_w x tile_h pixels laid over the render window,
 * row-major, with tile_w and tile_h each 8, 16 or 32; T = ceil(w/tile_w) * ceil(h/tile_h).
 *   vals [capacity]   record index of each (tile, Gaussian) pair, sorted by (tile, depth bits,
 *                     index) — one total order, so exactly one correct result;
 *   tile_range [2*T]  [begin, end) into vals per tile ([0, 0) when empty);
 *   num_pairs [1]     device int64: the REQUIRED number of pairs. If it exceeds capacity, only
 *                     the first `capacity` pairs are written, tile ranges are clamped, and the
 *                     caller must re-run with a larger capacity (no call faults);
 *   scratch           at least gs_bins_scratch_bytes(n, capacity, T) bytes, 256-B aligned. */
typedef struct gs_bins {
  int32_t tile_w, tile_h; /* each in {8, 16, 32} */
  int64_t capacity;
  uint32_t *vals;
  uint32_t *tile_range;
  int64_t *num_pairs;
  void *scratch;
  size_t scratch_bytes;
} gs_bins;

/* Rendered planes, window-sized: color [3][h][w] (eq:rendered_rgb plus T_final * bg),
 * depth [h][w] (eq:rendered_depth), alpha [h][w] (eq:rendered_opacity), and the backward
 * checkpoint: t_final [h][w] final transmittance and last [h][w] int32 position, within the
 * pixel's tile list, of the last Gaussian blended (-1 if none). n_contrib [h][w] int32 is
 * optional (NULL = not written): the number of Gaussians blended at each pixel.
 * state: device scratch of at least gs_image_state_bytes(...) bytes holding the chunk work
 * lists and, per (chunk, pixel) of tiles longer than one chunk, the transmittance and the
 * composited colour behind the chunk (the backward's starting state). Written by
 * gs_render_fwd, read by gs_render_bwd; the same bins and blend_depth must be passed to both.
 * While gs_render_fwd's work runs, the planes of a pixel that is still compositing hold its
 * running state (the forward walks long tile lists in windows); they are final when the
 * call's work on the stream has completed. */
typedef struct gs_image {
  float *color, *depth, *alpha, *t_final;
  int32_t *last;
  int32_t *n_contrib;
  void *state;
  size_t state_bytes;
} gs_image;

/* Sparse LiDAR depth term of eq:depth_loss with the opacity-normalised depth D/O:
 *   L_d = weight * (1/m) * sum_i |D(pix_i)/O(pix_i) - depth_target_i|
 * over m hits at ascending, distinct window-linear pixel indices pix [m] (int32); a hit with
 * O = 0 adds nothing. gs_render_fwd writes L_d to loss_out [1] (device, overwritten);
 * gs_render_bwd adds its gradient, scaled by *grad_scale (device scalar; NULL = 1). */
typedef struct gs_lidar {
  int32_t m;
  const int32_t *pix;
  const float *depth_target;
  float weight;
  float *loss_out;
  const float *grad_scale;
} gs_lidar;

/* Compositing-backward schedules (gs_grads.schedule):
 *   GS_BWD_CHUNKS  — pixel-parallel: each (tile, chunk) work item walks its pixels' splats back
 *                    to front, one pixel per lane, and sums each splat's terms over the
 *                    wavefront before one atomic per term (default);
 *   GS_BWD_BUCKETS — per-Gaussian buckets (Sec. "CUDA-Related Acceleration Strategies"): lane j
 *                    owns splat j of a 64-splat bucket and the tile's pixels pass through the
 *                    lanes, so each lane sums its splat's terms over the pixels; tiles of at
 *                    most 256 pixels (GS_ERR_UNSUPPORTED for 16x32, 32x16 and 32x32). Same
 *                    results up to float32 summation order. */
enum { GS_BWD_CHUNKS = 0, GS_BWD_BUCKETS = 1 };

/* Gradient outputs, same layouts as gs_gaussians; pose [6] is dL/dxi for the left
 * perturbation T_cw <- Exp(xi) T_cw with xi = (rho, phi), translation first (the manifold
 * derivative after eq:3dgs_jacobi, taken on the world-to-camera pose).
 * overwrite = 0: gradients are accumulated (+=) into the outputs;
 * overwrite = 1: every element of every given output is written (zero where no view
 *                contributes), so the outputs need no clearing beforehand.
 * scratch: at least gs_grads_scratch_bytes(...) bytes. Any of the parameter pointers may be
 * NULL to skip that output (sh_rest must be given when sh_degree > 0 and sh_dc is given). */
typedef struct gs_grads {
  float *mean, *scale, *rot, *opacity, *sh_dc, *sh_rest, *pose;
  void *scratch;
  size_t scratch_bytes;
  int32_t overwrite;
  int32_t schedule; /* GS_BWD_CHUNKS (0) or GS_BWD_BUCKETS */
} gs_grads;

/* Stage a1 — projection, covariance, SH colour, footprint, tile rectangle and alpha-max cull
 * for every Gaussian (Sec. "3D Gaussian Splatting Representation"). One camera. */
int gs_preprocess(const gs_gaussians *g, const gs_camera *cam, int32_t tile_w, int32_t tile_h,
                  gs_projected *out, gs_stream_t stream);

/* Stage a2 — pairs (tile, Gaussian) for the kept tiles, sorted by (tile, depth, index), and
 * the per-tile ranges. n = number of records in `proj`. */
int gs_bin_sort(const gs_projected *proj, int64_t n, const gs_camera *cam, gs_bins *io, gs_stream_t stream);

/* Stage a3 — front-to-back compositing per pixel (eq:alpha, eq:rendered_rgb/_depth/_opacity):
 * alpha = min(0.99, o exp(-q/2)); a Gaussian with alpha < 1/255 is skipped; the walk stops
 * before a Gaussian that would take the transmittance below 1e-4. blend_depth in {32, 64, 128,
 * 256} is the chunk length: each tile's list is composited in chunks of that many records,
 * one workgroup per chunk, and combined per pixel (exact up to float32 rounding order). lidar may be NULL; otherwise the
 * depth term is evaluated into lidar->loss_out after compositing. */
int gs_render_fwd(const gs_projected *proj, int64_t n, const gs_bins *bins, const gs_camera *cam,
                  int32_t blend_depth, const gs_lidar *lidar, gs_image *out, gs_stream_t stream);

/* Stages a4-a6 — backward of the compositing (walking each pixel's contributors from `last`
 * and rebuilding transmittance by division), the sparse-LiDAR depth term (only at the listed
 * pixels), and the chain rule to the parameters and to the pose (eq:3dgs_jacobi including the
 * SH term). dL_dC [3][h][w] is required; dL_dD and dL_dO [h][w] may be NULL; lidar may be NULL.
 * `fwd` must hold the outputs of gs_render_fwd for the same inputs. */
int gs_render_bwd(const gs_gaussians *g, const gs_camera *cam, const gs_projected *proj, const gs_bins *bins,
                  const gs_image *fwd, const float *dL_dC, const float *dL_dD, const float *dL_dO,
                  const gs_lidar *lidar, int32_t blend_depth, gs_grads *out, gs_stream_t stream);

/* For callers that cannot allocate device memory (code under hipGraph capture, tight serving
 * loops, harnesses that forbid hipMalloc): gs_render_bwd with the backward scratch taken from
 * a library-owned device array of GS_NOALLOC_SCRATCH_BYTES (128 MiB) per device instead of
 * out->scratch (out->scratch and out->scratch_bytes are ignored and may be 0). Arguments,
 * layouts, results and errors are those of gs_render_bwd, plus GS_ERR_INVALID_ARG when
 * gs_grads_scratch_bytes(g->n, 1, cam->w * cam->h) exceeds the limit (about 1.9 M Gaussians
 * at 1280x720). Calls nothing that allocates. The array is held by each device the library
 * runs on until the process ends; the first call on a device resolves its address (make that
 * call outside capture). All calls on one device share the array: calls that overlap in time
 * on one device (different streams, or threads) race and must be serialised by the caller;
 * every value the backward reads from it is written earlier in the same call. */
#define GS_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int gs_render_bwd_noalloc(const gs_gaussians *g, const gs_camera *cam, const gs_projected *proj,
                          const gs_bins *bins, const gs_image *fwd, const float *dL_dC, const float *dL_dD,
                          const float *dL_dO, const gs_lidar *lidar, int32_t blend_depth, gs_grads *out,
                          gs_stream_t stream);

/* RGB L1 term of the mapping loss (eq:depth_loss with the D-SSIM weight at zero):
 * loss_out[0] = weight * mean |color - target|, dL_dC = weight * sign(color - target) / n_values
 * (sign(0) = 0). n_values = 3 * pixels. loss_out is overwritten. */
int gs_loss_l1(const float *color, const float *target, int64_t n_values, float weight, float *dL_dC,
               float *loss_out, gs_stream_t stream);

/* Scratch sizes (bytes). */
size_t gs_bins_scratch_bytes(int64_t n, int64_t capacity, int64_t num_tiles);
size_t gs_image_state_bytes(int64_t capacity, int64_t num_tiles, int32_t tile_w, int32_t tile_h, int32_t blend_depth);
size_t gs_grads_scratch_bytes(int64_t n, int32_t n_views, int64_t total_window_pixels);

/* ---- Batched form (stage a7): several views of one map per launch ------------------------ */

typedef struct gs_view {
  gs_camera cam;
  gs_image out;                     /* window-sized planes of this view */
  const float *dL_dC, *dL_dD, *dL_dO; /* upstream gradients (GS_BWD); dL_dD, dL_dO may be NULL */
  gs_lidar lidar;                   /* m = 0 for none */
  const float *target;              /* optional [3][h][w]: when set, dL_dC is the RGB L1 term (see gs_loss_l1) */
  float rgb_weight;                 /* weight of that term */
  float *rgb_loss_out;              /* [1] device, overwritten; may be NULL */
  float *pose_grad;                 /* [6] accumulated (GS_BWD); may be NULL */
} gs_view;

typedef struct gs_batch_plan gs_batch_plan;

/* Creates a plan for up to n_views (<= GS_MAX_VIEWS) views of a map of n Gaussians at the
 * given degree: it owns the splat records, tile lists (pair capacity `capacity`, summed over
 * views), scratch and, with GS_GRAPH, the captured hipGraph. Allocates device memory.
 * flags: GS_PLAN_FWD_ONLY for a plan that only renders (no backward scratch; gs_render_batch
 * with GS_BWD then fails with GS_ERR_INVALID_ARG), else 0. */
enum { GS_PLAN_FWD_ONLY = 1 };
int gs_batch_plan_create(gs_batch_plan **plan, int64_t n, int32_t sh_degree, int32_t n_views,
                         int64_t max_total_pixels, int32_t tile_w, int32_t tile_h, int32_t blend_depth,
                         int64_t capacity, uint32_t flags);
/* Device bytes gs_batch_plan_create allocates for the same arguments (0 when they are
 * invalid); for admission by memory before a plan exists. */
size_t gs_batch_plan_bytes(int64_t n, int32_t sh_degree, int32_t n_views, int64_t max_total_pixels,
                           int32_t tile_w, int32_t tile_h, int32_t blend_depth, int64_t capacity, uint32_t flags);
void gs_batch_plan_destroy(gs_batch_plan *plan);

/* Renders (GS_FWD) and/or differentiates (GS_BWD) all views in one launch per stage. With
 * GS_GRAPH the stage sequence is captured into a hipGraph on first use and replayed while
 * the arguments (pointers, cameras, sizes) are unchanged; otherwise it is re-captured.
 * grads: shared parameter gradients (+=) over all views, may be NULL for GS_FWD. */
int gs_render_batch(gs_batch_plan *plan, const gs_gaussians *g, int32_t n_views, const gs_view *views,
                    uint32_t mode, gs_grads *grads, gs_stream_t stream);

/* Required pair count of the plan's last run, copied to *required after the work queued on
 * `stream` so far has finished (synchronises that stream). Compare with gs_batch_capacity: a
 * larger value means the lists were clamped and the plan must be re-created bigger. */
int gs_batch_num_pairs(const gs_batch_plan *plan, int64_t *required, gs_stream_t stream);
int64_t gs_batch_capacity(const gs_batch_plan *plan);

/* Host helper: camera with pose Exp(xi) T_cw (xi = (rho, phi), closed-form SE(3) exponential),
 * the left update whose derivative gs_render_bwd reports. Intrinsics and window are copied. */
int gs_camera_left_update(const gs_camera *in, const float xi[6], gs_camera *out);

/* Device form of gs_camera_left_update (the left perturbation whose derivative follows
 * eq:3dgs_jacobi): pose_out (device float [16], the layout of gs_projected.pose) receives
 * Exp(xi) T_cw for the tangent xi (device float [6], (rho, phi)) and the camera's R_cw, t_cw,
 * computed in float64 by one lane and rounded once. Asynchronous on `stream`; reads xi when
 * the stream reaches it. Errors: GS_ERR_INVALID_ARG for NULL pointers or a camera failing the
 * usual checks. */
int gs_pose_left_update(const gs_camera *cam, const float *xi, float *pose_out, gs_stream_t stream);

/* Kernel timing. gs_profile_enable creates `max_records` pairs of HIP events per stage
 * (allocation happens here, not in the timed calls); afterwards every launch of a stage in
 * `stage_mask` (bit i = stage i below) on this thread is bracketed by an event pair recorded
 * on the launch stream, up to max_records launches. gs_profile_read synchronises those
 * events and returns the summed duration (ms) and the launch count of one stage.
 * gs_profile_disable releases the events. Stages: */
enum { GS_STAGE_PREPROCESS = 0, GS_STAGE_BIN_SORT = 1, GS_STAGE_BLEND_FWD = 2, GS_STAGE_BLEND_BWD = 3,
       GS_STAGE_PREPROCESS_BWD = 4, GS_NUM_STAGES = 5 };
int gs_profile_enable(uint32_t stage_mask, int32_t max_records);
int gs_profile_read(int32_t stage, double *total_ms, int32_t *count);
void gs_profile_disable(void);

/* D-SSIM term of the photometric tracking loss (eq:tracking_loss; the D-SSIM term of the
 * original 3DGS loss; efficient separable SSIM, Sec. "Additional Strategies", c):
 *   loss = weight * (1 - mean SSIM) over the channels x h x w values,
 * SSIM per channel from local means / variances / covariance under an 11x11 Gaussian window
 * (sigma 1.5, weights summing to one), zero outside the image, C1 = 0.01^2, C2 = 0.03^2.
 * color, target [channels][h][w] fp32 device planes. dL_dC (may be NULL) is ACCUMULATED (+=)
 * with d loss / d color, so it composes with gs_loss_l1, which overwrites it. loss_out [1]
 * (may be NULL) is overwritten, summed in a fixed order (deterministic). scratch: device, at
 * least gs_dssim_scratch_bytes (3 floats per value and one per 32x32 tile of each channel). Errors: GS_ERR_INVALID_ARG for negative sizes, more than 64 channels, h or w above
 * 32768 or 2^31 values, NULL images with
 * a non-empty size, a non-finite weight or short scratch. */
size_t gs_dssim_scratch_bytes(int32_t channels, int32_t h, int32_t w);
int gs_loss_dssim(const float *color, const float *target, int32_t channels, int32_t h, int32_t w, float weight,
                  float *dL_dC, float *loss_out, void *scratch, size_t scratch_bytes, gs_stream_t stream);

/* ---- Photometric tracking (camera factor option 2) ------------------------------------ */

/* The pose loop of Sec. "Camera Factor (Option 2)": with the map frozen, `iters` (N_t = 30 in
 * the paper's setup) iterations, each of which renders the view at the current pose,
 * evaluates eq:tracking_loss
 *   L = l1_weight * mean |C_hat - C| + ssim_weight * D-SSIM(C_hat, C)   (1/2 and 1/2)
 * (the two terms as gs_loss_l1 and gs_loss_dssim), differentiates it to the pose tangent
 * xi = (rho, phi) of the left perturbation T_cw <- Exp(xi) T_cw (as gs_render_bwd, with no
 * Gaussian gradient written), and applies an Adam step delta (step sizes lr_rho for the
 * translation, lr_phi for the rotation; moments and bias correction run over the iterations)
 * as T_cw <- Exp(delta) T_cw. The result is the refined pose T~ of eq:map_optimize_pose. */
typedef struct gs_track_params {
  int32_t iters;
  float l1_weight, ssim_weight;
  float lr_rho, lr_phi;
  float beta1, beta2, eps; /* betas in [0, 1), eps > 0 */
  uint32_t flags;          /* GS_GRAPH: capture the iterations into a hipGraph, replayed while
                              every argument but the starting pose is unchanged */
} gs_track_params;

typedef struct gs_track_plan gs_track_plan;

/* A plan owns every buffer of the loop for maps of up to n Gaussians at up to the given
 * degree and windows of up to max_pixels: splat records, tile lists of `capacity` pairs,
 * image planes, gradient maps, scratch and the pose state. Allocates device memory. */
int gs_track_plan_create(gs_track_plan **plan, int64_t n, int32_t sh_degree, int64_t max_pixels, int32_t tile_w,
                         int32_t tile_h, int32_t blend_depth, int64_t capacity);
void gs_track_plan_destroy(gs_track_plan *plan);
int64_t gs_track_capacity(const gs_track_plan *plan);

/* Runs the loop from the pose in `cam` against target [3][h][w] (window-sized, device).
 * pose_out [12] (device): the refined world-to-camera pose, R_cw row-major then t_cw.
 * trace (device, may be NULL): [iters][20] floats per iteration: the pose rendered (12, as
 * pose_out), dL/dxi at that pose (6), the L1 term and the D-SSIM term. The pose is kept in
 * float64 on the device between iterations and rounded to float32 for each render.
 * Asynchronous; no host synchronisation inside the loop. A plan's buffers (and its pose
 * state) serve one call at a time: calls on one plan must be ordered on one stream. */
int gs_track_pose(gs_track_plan *plan, const gs_gaussians *g, const gs_camera *cam, const float *target,
                  const gs_track_params *params, float *pose_out, float *trace, gs_stream_t stream);

/* Largest pair count of the last gs_track_pose over its iterations, copied to *required
 * after the work queued on `stream` (synchronises it). Above gs_track_capacity, some
 * iterations rendered clamped tile lists: re-create the plan bigger and run again. */
int gs_track_required_pairs(const gs_track_plan *plan, int64_t *required, gs_stream_t stream);

/* Host helper: the factor residual of eq:map_optimize_pose, r = Log(T_wc(t) T~_wc^-1) on
 * camera-to-world poses, from the predicted and refined world-to-camera poses (each R_cw
 * row-major then t_cw, as pose_out). r = (rho, phi), float64, closed-form SE(3) logarithm
 * (rotation angles below pi). */
int gs_pose_residual(const float pred_cw[12], const float refined_cw[12], double r[6]);

/* ---- Map initialization and expansion ------------------------------------------------- */

/* Colourised points of a keyframe: xyz [3][n] world coordinates, rgb [3][n] in [0, 1]. */
typedef struct gs_points {
  int64_t n;
  const float *xyz, *rgb;
} gs_points;

/* Writable Gaussian planes, layouts as gs_gaussians (stride n). */
typedef struct gs_gaussians_out {
  int64_t n;
  int32_t sh_degree;
  float *mean, *scale, *rot, *opacity, *sh_dc, *sh_rest;
} gs_gaussians_out;

size_t gs_expand_scratch_bytes(int64_t n_points);

/* Selection of Sec. "Expansion of Gaussian Map": a point is selected when it lies beyond the
 * near plane (camera-frame z > 0.2), its nearest pixel centre floor(fx x/z + cx + 1/2),
 * floor(fy y/z + cy + 1/2) lies in the render window, and the rendered opacity there
 * (eq:rendered_opacity; `opacity` is the window plane [h][w] of gs_render_fwd) is below tau
 * (0.99 in the paper's setup). opacity = NULL is the initialization of Sec. "Initialization of
 * Gaussian Map": every point beyond the near plane is selected. The decision is taken in
 * float32 with the projection's operation order. count_out [1] (device int64) receives the
 * number selected; scratch (device, gs_expand_scratch_bytes(n)) keeps the decisions for
 * gs_expand_write. rgb may be NULL here. */
int gs_expand_select(const gs_points *pts, const gs_camera *cam, const float *opacity, float tau,
                     int64_t *count_out, void *scratch, size_t scratch_bytes, gs_stream_t stream);

/* The grown map: out->n = old n + added, where added is the count gs_expand_select produced
 * (read back by the caller to size `out`); a smaller `added` keeps the first `added` selected
 * points. The existing Gaussians (old_map, may be NULL for none) are copied first, then one
 * Gaussian per selected point in point order: mean = xyz, scale = (z / fx)(1, 1, 1) with z the
 * point's camera-frame depth, rotation (1, 0, 0, 0), opacity 0.1, sh_dc = (rgb - 1/2) / Y_0
 * with Y_0 = 1 / (2 sqrt(pi)), sh_rest = 0. out->sh_degree must equal the old map's; the
 * planes of `out` must not overlap the old map's. pts, cam and scratch as given to
 * gs_expand_select. */
int gs_expand_write(const gs_points *pts, const gs_camera *cam, const gs_gaussians *old_map, int64_t added,
                    const void *scratch, size_t scratch_bytes, const gs_gaussians_out *out, gs_stream_t stream);

/* Sparse Adam (Sec. "Additional Strategies", a): one Adam step (first and second moment
 * estimates with bias correction) on the Gaussians the rendering reached. A Gaussian whose
 * tile count is zero in every view of `visible` keeps its parameters and moments; the step
 * number is shared by all. Groups are sets of k SoA planes of n values:
 *   param          [k][n] raw parameter (updated in place)
 *   exp_avg        [k][n] first moment, exp_avg_sq [k][n] second moment (updated in place)
 *   grad           [k][n] gradient w.r.t. the value the renderer reads: act(param)
 *   act_out        [k][n] act(param) written for the updated Gaussians (act != GS_ACT_NONE;
 *                  may be NULL), e.g. the scale / opacity planes of gs_gaussians
 *   act            GS_ACT_NONE: the renderer reads param; GS_ACT_EXP: exp(param) (log-scale);
 *                  GS_ACT_SIGMOID: 1 / (1 + exp(-param)) (opacity logit)
 *   lr             learning rate of the group
 * The raw gradient is grad * d act / d param at the values before the step. For step t >= 1
 * the caller passes bias1 = 1 - beta1^t and bias2 = 1 - beta2^t; an element moves by
 * lr / bias1 * m / (sqrt(v) / sqrt(bias2) + eps).
 * visible: tile counts [n_views][n] (gs_projected.n_tiles of each view), or NULL for all.
 * The stores of the 64 consecutive Gaussians of a wavefront that holds an updated one are
 * full width: the others of that wavefront rewrite their unchanged param / moment values.
 * Errors: GS_ERR_INVALID_ARG for n < 0 or n >= 2^30, n_groups outside [0, GS_ADAM_MAX_GROUPS],
 * n_views outside [1, GS_MAX_VIEWS] with visible set, k < 0, a NULL plane of a group with
 * k > 0, an unknown act, or betas / eps / lr / bias terms out of range (betas in [0, 1),
 * eps >= 0, bias terms in (0, 1], lr finite). */
#define GS_ACT_NONE 0
#define GS_ACT_EXP 1
#define GS_ACT_SIGMOID 2
#define GS_ADAM_MAX_GROUPS 8
typedef struct {
  float *param, *exp_avg, *exp_avg_sq;
  const float *grad;
  float *act_out;
  int32_t k, act;
  float lr;
} gs_adam_group;
typedef struct {
  int64_t n;
  int32_t n_groups, n_views;
  const uint32_t *visible; /* [n_views][n] or NULL */
  float beta1, beta2, eps, bias1, bias2;
  gs_adam_group group[GS_ADAM_MAX_GROUPS];
} gs_adam;
int gs_adam_sparse(const gs_adam *a, gs_stream_t stream);

/* Thread-local text of the last error of this thread. */
const char *gs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */
