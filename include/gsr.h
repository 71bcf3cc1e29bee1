/*
 * gsr.h -- C ABI of the MI355X (gfx950) differentiable tile-based Gaussian
 * splatting renderer: the rendering hot path of GS-SLAM's tracking and
 * mapping loops (Yan et al., "GS-SLAM: Dense Visual SLAM with 3D Gaussian
 * Splatting", arXiv 2311.11700).
 *
 * Method (paper references):
 *   - Scene: Gaussians with mean, covariance R S S^T R^T (Eq. 1-2, rotation
 *     from a real-first quaternion, supplement eq. q2R), opacity, and either
 *     an RGB colour or degree-1 spherical-harmonic coefficients evaluated in
 *     the viewing direction (Sec. 3.1).
 *   - Projection: Sigma' = J W Sigma W^T J^T (Eq. 3) plus a low-pass term;
 *     centre m = K X_c / z, depth d = z (Sec. 3.1, Sec. 3.3).
 *   - Binning: 16x16 tiles; a Gaussian covers the tiles of the bounding box of
 *     its cutoff_sigma ellipse; tile lists sorted by (tile, float32 depth bits,
 *     Gaussian index).
 *   - Compositing: front-to-back alpha blending of colour (Eq. 4) and depth
 *     (Eq. 5), final transmittance T_final = 1 - cumulative opacity (Sec. 3.2).
 *   - Backward: gradients of the blend (supplement eq. grad_depth and its
 *     colour analogue), chained through the projection to every Gaussian
 *     parameter and to the camera pose (Eq. 11 and supplement Sec. A; the
 *     Sigma' path of the pose gradient is kept unless GSR_PAPER_POSE_APPROX).
 *   - Loss: weighted L1 on colour and depth (Eq. 6, Eq. 10).
 *   - Map expansion: the adding step (Eq. 8, new Gaussians at unreliable
 *     pixels) and the deleting step (Eq. 9, opacity decay) of Sec. 3.2.
 *
 * Conventions
 *   - All arrays are caller-owned DEVICE memory unless marked HOST.
 *   - Pixel (x, y) has its centre at integer coordinates (x, y).
 *   - Views are concatenated: view v's pixels start at pixel offset
 *     P_v = sum_{u<v} W_u H_u.  Colour images are planar per view:
 *     rgb[3 * P_v + c * H_v * W_v + y * W_v + x].  depth, T_final, last and the
 *     per-pixel upstream gradients use [P_v + y * W_v + x].
 *   - Gradient outputs ACCUMULATE (+=): the caller zeroes them before the
 *     first call; batched views and repeated calls sum.
 *   - Functions return a gsr_status and never throw.  Calls on one context
 *     are not thread-safe; use one context per host thread.
 *   - Nothing on the render path allocates device memory: scratch lives in the
 *     caller's workspace, sized by gsr_plan().
 */
#ifndef GSR_H
#define GSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gsr_ctx gsr_ctx;
/* A hipStream_t passed as an opaque pointer (NULL = the null stream). */
typedef void *gsr_stream;

typedef enum {
  GSR_OK = 0,
  GSR_E_INVALID = -1,     /* bad argument: null pointer, size mismatch with the plan, ... */
  GSR_E_CAPACITY = -2,    /* the tile-pair buffer was too small: see gsr_required_pairs() */
  GSR_E_HIP = -3,         /* a HIP runtime call failed: see gsr_last_error() */
  GSR_E_UNSUPPORTED = -4, /* configuration not supported (e.g. a view wider than 65535 px) */
  GSR_E_STATE = -5        /* call out of order (no plan, workspace not filled by a forward) */
} gsr_status;

/* One camera (80 bytes, DEVICE array [n_views]).  Pinhole intrinsics in
 * pixels; world->camera pose X_c = R X + t (R row-major).  width/height must
 * equal the sizes given to gsr_plan() for this view. */
typedef struct {
  float fx, fy, cx, cy;
  float R[9];
  float t[3];
  int32_t width, height;
  int32_t _pad[2];
} gsr_camera;

/* The Gaussian set (Eq. 1-2), structure of arrays, float32, DEVICE:
 *   mean [n][3], log_scale [n][3] (scale = exp), quat [n][4] (w, x, y, z;
 *   normalised inside), opacity_logit [n] (opacity = sigmoid), rgb [n][3].
 *   mask [n] (nullable, uint8): 0 excludes a Gaussian (coarse-to-fine
 *   selection of reliable Gaussians, Eq. 12).
 *   sh [n][4][3] (nullable): degree-1 spherical-harmonic colour, 12
 *   coefficients per Gaussian (Sec. 3.1).  When set, the colour of Gaussian
 *   i in a view is, per channel c, sum_k Y_k(d) sh[i][k][c] with d the unit
 *   direction from the camera centre -R^T t to the mean and the real
 *   harmonics Y_0 = 1/(2 sqrt(pi)), (Y_1, Y_2, Y_3) = sqrt(3/(4 pi)) (d_y,
 *   d_z, d_x); rgb is then not read (may be NULL).  No offset, no clamp.
 * Non-finite parameters and zero quaternions cull the Gaussian. */
typedef struct {
  int64_t n;
  const float *mean, *log_scale, *quat, *opacity_logit, *rgb;
  const uint8_t *mask;
  const float *sh;
} gsr_gaussians;

enum {
  /* Every Gaussian covers every tile of every view (finite-difference mode:
   * together with alpha_min = T_min = 0 and alpha_max = 1 the image is a
   * smooth function of the parameters). */
  GSR_FULL_RECT = 1u << 0,
  /* Backward: produce gradients for the Gaussian parameters. */
  GSR_GAUSS_GRAD = 1u << 1,
  /* Backward: produce the se(3) pose gradient of every view. */
  GSR_POSE_GRAD = 1u << 2,
  /* Pose gradient through the projected centre and depth only, dropping
   * the Sigma' term as the paper does for speed (Sec. 3.3, supplement). */
  GSR_PAPER_POSE_APPROX = 1u << 3,
  /* Fused step and backward: write the gradients (and the fused step's
   * loss) instead of adding them to the caller's buffers, so the caller
   * need not clear them between steps. */
  GSR_GRAD_OVERWRITE = 1u << 4
};

/* Renderer constants.  The paper is silent on them; gsr_default_config()
 * returns the values of the 3DGS rasteriser the paper extends:
 * alpha_min 1/255, alpha_max 0.99, T_min 1e-4, cutoff_sigma 3, z_near 0.2 m,
 * lowpass 0.3 px^2, bg 0, flags GSR_GAUSS_GRAD | GSR_POSE_GRAD, fov_guard 1.3.
 * Calls reject alpha_min outside [0, 1], alpha_max outside (0, 1], a
 * negative T_min, cutoff_sigma <= 0 and a negative or non-finite fov_guard.
 *
 * fov_guard g > 0 limits the Jacobian of Eq. 3 (not the projected centre):
 * x/z and y/z enter J clamped to +-g W/(2 fx) and +-g H/(2 fy), so a
 * Gaussian just beyond the near plane far to the side of the view keeps a
 * bounded footprint instead of a linearisation that smears it over the whole
 * image; the backward differentiates the clamped function.  g = 0 uses Eq. 3
 * as printed. */
typedef struct {
  float alpha_min, alpha_max, T_min, cutoff_sigma, z_near, lowpass;
  float bg[3];
  uint32_t flags;
  float fov_guard;
} gsr_config;

/* Forward outputs, DEVICE (any pointer may be NULL to skip that output):
 * rgb [3 * sum HW] float, depth / T_final [sum HW] float, last [sum HW] int32
 * (1 + position in the tile list of the pixel's last blended Gaussian),
 * loss [sum HW] float: the pixel's own term of the L1 loss (written by the
 * fused step only, before any loss cap; 0 where pixel_mask is 0). */
typedef struct {
  float *rgb, *depth, *T_final;
  int32_t *last;
  float *loss;
} gsr_images;

/* Gradient outputs, DEVICE, accumulated (+=).  d_* match the Gaussian
 * arrays; d_pose [n_views][6] = (rho_x, rho_y, rho_z, phi_x, phi_y, phi_z):
 * the derivative w.r.t. a left perturbation T_cw <- Exp(xi) T_cw at xi = 0.
 * With spherical-harmonic colour d_sh [n][4][3] receives the coefficient
 * gradient and d_rgb is not written (may be NULL); the viewing direction
 * adds to d_mean and d_pose.  Pointers may be NULL when the matching flag
 * is off. */
typedef struct {
  float *d_mean, *d_log_scale, *d_quat, *d_opacity_logit, *d_rgb;
  float *d_pose;
  float *d_sh;
} gsr_grads;

/* Tuning parameters (picked by gsr_autotune, or set by hand). */
typedef struct {
  int32_t blocks_per_cu;   /* persistent rasteriser: resident blocks per CU (1..8) */
  int32_t tiles_per_pop;   /* tiles a block takes from the work queue at a time (1..8) */
  int32_t lpt_order;       /* 1: process tiles longest first, by the durations the previous fused step on
                              the workspace recorded (index order until one has); 0: index order */
  int32_t batch;           /* records the fused rasteriser stages in LDS per forward round: 64, 128, 192
                              or 256 (0: 192); fewer leave room for more resident blocks per CU */
} gsr_tuning;

gsr_config gsr_default_config(void);
const char *gsr_status_string(gsr_status s);
/* Text of the last error on this context (never NULL). */
const char *gsr_last_error(const gsr_ctx *ctx);

/* Create a context on HIP device `device` (owns a few KB of device memory for
 * the view table and a pinned host word; no other state).  The first call on
 * a device also resolves the address of that device's static scratch (see
 * gsr_render_l1_fused_noalloc). */
gsr_status gsr_create(int device, gsr_ctx **out);
void gsr_destroy(gsr_ctx *ctx);

/* Plan a workload: n Gaussians rendered into n_views views of sizes
 * wh_host[v] = (width, height) (HOST array [n_views][2]), with room for
 * pair_capacity (tile, Gaussian) pairs.  Writes the workspace size in bytes
 * the render calls need.  Synchronous; not on the hot path. */
gsr_status gsr_plan(gsr_ctx *ctx, int64_t n, int n_views, const int32_t *wh_host,
                    int64_t pair_capacity, size_t *workspace_bytes);

/* Forward render (Eq. 3-5) of every planned view.  `workspace` (DEVICE,
 * >= workspace_bytes, 256-byte aligned) keeps the projected Gaussians, the
 * sorted tile lists and per-pixel state for gsr_render_backward.
 * Asynchronous: a pair-capacity overflow is recorded on the device and
 * reported by gsr_check_overflow() (with gsr_required_pairs() telling the
 * capacity to plan for); after an overflow the outputs are undefined. */
gsr_status gsr_render_forward(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams,
                              int n_views, const gsr_config *cfg, void *workspace,
                              size_t workspace_bytes, const gsr_images *out, gsr_stream stream);

/* Generation of the last successful gsr_render_forward on this context: 1,
 * 2, ... in call order (0 before the first).  A caller that keeps several
 * forwards in flight (an autograd graph) records it after each forward and
 * passes it to gsr_render_backward. */
int64_t gsr_forward_generation(const gsr_ctx *ctx);

/* Backward of a forward on this workspace: upstream gradients g_rgb
 * [3 * sum HW], g_depth [sum HW], g_T (nullable) [sum HW] w.r.t. the colour,
 * depth and final-transmittance outputs.  forward_generation must be the
 * gsr_forward_generation() value of the forward whose state the workspace
 * holds, i.e. of the last forward on this context, on this workspace, with no
 * fused step, autotune or plan since; otherwise GSR_E_STATE (the state of an
 * earlier forward has been overwritten).  Accumulates into `grads` according
 * to cfg->flags.  Asynchronous. */
gsr_status gsr_render_backward(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams,
                               int n_views, const gsr_config *cfg, void *workspace,
                               size_t workspace_bytes, int64_t forward_generation, const float *g_rgb,
                               const float *g_depth, const float *g_T, const gsr_grads *grads,
                               gsr_stream stream);

/* Weighted L1 loss (Eq. 6 / Eq. 10) and its gradient w.r.t. the rendered
 * images: loss = w_rgb sum m |C - C*| + w_depth sum m [D* > 0] |D - D*| over
 * all views' pixels with pixel_mask (nullable uint8, 0 = ignore) != 0;
 * sign(0) = 0.  w_rgb, w_depth >= 0.  loss_cap (DEVICE float [n_views],
 * nullable): a pixel whose own loss term exceeds its view's cap is ignored
 * (no loss, zero gradient) -- the tracking rule that drops pixels with more
 * than ten times the median loss (implementation details of the paper; see
 * gsr_loss_median).  Writes (overwrites) g_rgb / g_depth; ADDS the loss into
 * *loss (DEVICE float).  Asynchronous. */
gsr_status gsr_l1_loss_grad(gsr_ctx *ctx, const float *rgb, const float *depth,
                            const float *target_rgb, const float *target_depth,
                            const uint8_t *pixel_mask, float w_rgb, float w_depth,
                            const float *loss_cap, float *g_rgb, float *g_depth, float *loss,
                            gsr_stream stream);

/* One training step of the renderer in a single call: forward, L1 loss and
 * its gradient (as gsr_l1_loss_grad, loss_cap included), and backward, with
 * the per-tile forward, loss gradient and backward fused in one persistent
 * kernel.  Images in `out` are optional (NULL struct or NULL members skip
 * them; out->loss receives every pixel's own loss term before the cap).
 * ADDS the loss into *loss.  Asynchronous: a pair-capacity overflow is
 * recorded on the device and reported by gsr_check_overflow().  The
 * backward's per-entry sums over a tile's pixels run on the bf16 matrix
 * cores with every FP32 operand split into a high and a low bf16 half
 * (relative error below 2^-16 per operand, FP32 accumulation), as in
 * gsr_render_backward. */
gsr_status gsr_render_l1_fused(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams,
                               int n_views, const gsr_config *cfg, const float *target_rgb,
                               const float *target_depth, const uint8_t *pixel_mask, float w_rgb,
                               float w_depth, const float *loss_cap, void *workspace,
                               size_t workspace_bytes, const gsr_images *out, const gsr_grads *grads,
                               float *loss, gsr_stream stream);

/* Size of the static scratch behind gsr_render_l1_fused_noalloc: 64 MiB of
 * device memory per GPU the library runs on, held until the process ends. */
#define GSR_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* gsr_render_l1_fused without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP-graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The workspace is a static device array of
 * GSR_NOALLOC_SCRATCH_BYTES inside the library (one per GPU, its address
 * resolved once per device by gsr_create); the call itself allocates nothing
 * and issues no memset.  Same kernels, arguments, outputs and asynchronous
 * semantics as gsr_render_l1_fused.  GSR_E_INVALID when the plan's workspace
 * (gsr_plan's workspace_bytes) exceeds GSR_NOALLOC_SCRATCH_BYTES.
 * Every call on a GPU shares that GPU's array and leaves its state in it:
 * calls that overlap on one GPU (two streams, two contexts, two host threads)
 * race and give undefined results; serialise them.  A pair-capacity
 * overflow is read with gsr_check_overflow(ctx, NULL, stream). */
gsr_status gsr_render_l1_fused_noalloc(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams,
                                       int n_views, const gsr_config *cfg, const float *target_rgb,
                                       const float *target_depth, const uint8_t *pixel_mask, float w_rgb,
                                       float w_depth, const float *loss_cap, const gsr_images *out,
                                       const gsr_grads *grads, float *loss, gsr_stream stream);

/* Capture gsr_render_l1_fused with these exact arguments (pointers and
 * scalar values are baked in; buffer CONTENTS may change between launches)
 * into a HIP graph owned by the context, replacing any earlier capture. */
gsr_status gsr_graph_capture(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams,
                             int n_views, const gsr_config *cfg, const float *target_rgb,
                             const float *target_depth, const uint8_t *pixel_mask, float w_rgb,
                             float w_depth, const float *loss_cap, void *workspace,
                             size_t workspace_bytes, const gsr_images *out, const gsr_grads *grads,
                             float *loss, gsr_stream stream);
/* Launch the captured graph on `stream` (asynchronous). */
gsr_status gsr_graph_launch(gsr_ctx *ctx, gsr_stream stream);

/* Synchronise `stream`, then report GSR_E_CAPACITY if any call since the
 * last check overflowed the pair buffer of this workspace (NULL: the static
 * scratch of gsr_render_l1_fused_noalloc on the context's device). */
gsr_status gsr_check_overflow(gsr_ctx *ctx, void *workspace, gsr_stream stream);
/* Pair count of the last overflowing call (0 if none). */
int64_t gsr_required_pairs(const gsr_ctx *ctx);
/* Synchronise `stream` and return the number of (tile, Gaussian) pairs the
 * last forward on `workspace` produced: one per tile of each visible
 * Gaussian's 3-sigma rectangle, including the pairs whose tile lies outside
 * the Gaussian's alpha support (those are dropped by the pair sort and not
 * rendered). */
int64_t gsr_pair_count(gsr_ctx *ctx, void *workspace, gsr_stream stream);

/* DEVICE pointers into the workspace, for inspection after a forward:
 * tile_ranges [total_tiles][2] int32 (start, end) into the sorted lists,
 * sorted_ids [pairs] uint32 = view * n + gaussian index.  Tiles are numbered
 * view after view, row-major within a view. */
gsr_status gsr_debug_tiles(gsr_ctx *ctx, void *workspace, const int32_t **tile_ranges,
                           const uint32_t **sorted_ids, int64_t *total_tiles);

/* Tuning of the fused rasteriser. */
gsr_status gsr_get_tuning(const gsr_ctx *ctx, gsr_tuning *out);
gsr_status gsr_set_tuning(gsr_ctx *ctx, const gsr_tuning *t);
/* Time candidate tunings on this workload (same arguments as
 * gsr_render_l1_fused; gradients and loss are written by the trial runs, so
 * the caller re-zeroes them afterwards): every work order, blocks per CU and
 * tiles per pop at batch 192, then the other batch sizes at the best of
 * those (one of them only if 2 % faster); keep the fastest in the context
 * and return it.  `reps` timed
 * launches per candidate. */
gsr_status gsr_autotune(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cams, int n_views,
                        const gsr_config *cfg, const float *target_rgb, const float *target_depth,
                        const uint8_t *pixel_mask, float w_rgb, float w_depth, void *workspace,
                        size_t workspace_bytes, const gsr_grads *grads, float *loss, int reps,
                        gsr_tuning *best, gsr_stream stream);

/* Loss cap for outlier pixels (implementation details of the paper: a
 * tracking pixel whose loss exceeds ten times the median loss is ignored).
 * For every view of the plan: cap_out[v] = factor * the lower median (the
 * element of rank floor((m - 1) / 2) in ascending order) of px_loss over the
 * view's m pixels with pixel_mask != 0 (all pixels if pixel_mask is NULL);
 * +inf when m = 0.  px_loss (DEVICE float [sum HW], e.g. gsr_images.loss of
 * a fused step) is compared as non-negative floats: negative values and -0
 * count as 0, NaN above +inf.  The selection is exact (radix select on the
 * float bits, one block per view).  cap_out is DEVICE float [n_views], the
 * loss_cap argument of the next step.  Asynchronous. */
gsr_status gsr_loss_median(gsr_ctx *ctx, const float *px_loss, const uint8_t *pixel_mask, float factor,
                           float *cap_out, gsr_stream stream);

/* Reliable-Gaussian selection for the fine tracking stage (Eq. 12, Sec. 3.3):
 * each Gaussian's centre is projected with the (coarse) pose `cam` (DEVICE,
 * one gsr_camera); when it lands in front of the camera (z > z_near) on a
 * pixel inside the image whose observed depth D (depth_obs, DEVICE
 * [height][width] float, 0 = no reading) is valid, the Gaussian is kept only
 * if |D - z| <= eps, z being the camera-frame depth of its centre.
 * Gaussians that project outside the image, behind the near plane or onto a
 * missing reading are kept; Gaussians already excluded by g->mask stay
 * excluded.  The pixel is the one nearest to the projected centre
 * (floor(u + 0.5), floor(v + 0.5)); the projection is evaluated in FP64.
 * Writes mask_out[n] (DEVICE uint8, 1 = selected).  Asynchronous. */
gsr_status gsr_select_reliable(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cam,
                               const float *depth_obs, int width, int height, float eps, float z_near,
                               uint8_t *mask_out, gsr_stream stream);

/* Adaptive expansion of the map (Sec. 3.2).
 *
 * Writable Gaussian arrays that the adding step appends to (DEVICE,
 * `capacity` rows each, same layouts as gsr_gaussians; quat 16-byte
 * aligned): rgb [capacity][3] and/or, for a map with spherical-harmonic
 * colour, sh [capacity][4][3] (either may be NULL, not both). */
typedef struct {
  float *mean, *log_scale, *quat, *opacity_logit, *rgb;
  float *sh;
} gsr_gaussians_out;

/* Adding-step parameters: tau_T (cumulative-opacity threshold) and tau_D
 * (depth-error threshold, metres) of Eq. 8; the new Gaussians' isotropic
 * scale is scale_factor * D / sqrt(fx fy) (the spacing of back-projected
 * neighbouring pixels at depth D) and their opacity logit
 * opacity_logit_init (the predefined initial opacity of Eq. 7). */
typedef struct {
  float tau_T, tau_D, scale_factor, opacity_logit_init;
} gsr_expand_params;

/* Adding step (Eq. 8) over every planned view: a pixel is unreliable when it
 * has a depth reading (depth_obs > 0) and its cumulative opacity
 * 1 - T_final is below tau_T or |depth_obs - depth| exceeds tau_D (FP64
 * decisions on the float32 inputs).  Each unreliable pixel (x, y) of view v,
 * in pixel order (views in order, rows top to bottom, left to right),
 * becomes a new Gaussian (Eq. 7): mean = R^T (X_c - t) with
 * X_c = D ((x - cx) / fx, (y - cy) / fy, 1) and D = depth_obs, all three
 * log-scales log(scale_factor D / sqrt(fx fy)), quaternion (1, 0, 0, 0),
 * opacity logit opacity_logit_init, rgb = rgb_obs at the pixel; in a map
 * with degree-1 SH colour, sh = (rgb_obs / Y_0, 0, 0, 0) per channel (the
 * observed colour from every direction; Y_0 = 1 / (2 sqrt(pi))).  The k-th
 * new Gaussian is written at index n + k of `out` when n + k < capacity.
 * Inputs use the concatenated image layouts of the plan's views (T_final and
 * depth as a forward writes them; depth_obs [sum HW]; rgb_obs [3 * sum HW]);
 * cams DEVICE [n_views].  Writes *count (DEVICE int64) = the number of
 * unreliable pixels (new Gaussians wanted: more than capacity - n means the
 * arrays were too small and only the first capacity - n were written) and,
 * when pixel_flag (DEVICE uint8 [sum HW]) is not NULL, each pixel's
 * decision.  Uses only the workspace's adding-step scratch, so a forward's
 * state in the same workspace is kept.  Asynchronous. */
gsr_status gsr_expand_add(gsr_ctx *ctx, const gsr_camera *cams, int n_views, const float *T_final, const float *depth,
                          const float *depth_obs, const float *rgb_obs, const gsr_expand_params *params,
                          void *workspace, size_t workspace_bytes, int64_t n, int64_t capacity,
                          const gsr_gaussians_out *out, uint8_t *pixel_flag, int64_t *count, gsr_stream stream);

/* Deleting step (Eq. 9) for one view `cam` (DEVICE, one gsr_camera) with its
 * observed depth depth_obs (DEVICE [height][width], 0 = no reading).  A
 * Gaussian is visible when its centre lies beyond z_near and projects to a
 * pixel of the image (the nearest one, (floor(u + 0.5), floor(v + 0.5)))
 * with a reading D; the observed surface point of that pixel lies on the
 * Gaussian's ray at D / z times its camera-frame centre X_c, and when it lies
 * more than gamma beyond the Gaussian, (D - z) |X_c| / z > gamma (the
 * Gaussian floats in front of the surface), the opacity is scaled by eta:
 * sigmoid(Lambda') = eta sigmoid(Lambda), 0 < eta <= 1.  The printed
 * condition D - dist(X_i, P_uv) > gamma is read as this signed distance.
 * Writes every Gaussian's logit to opacity_logit_out (DEVICE [n]; may alias
 * g->opacity_logit) and, when decayed (DEVICE uint8 [n]) is not NULL, 1 for
 * the decayed ones.  Gaussians excluded by g->mask are left unchanged.
 * Evaluated in FP64; asynchronous; no plan needed. */
gsr_status gsr_expand_delete(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_camera *cam, const float *depth_obs,
                             int width, int height, float gamma, float eta, float z_near, float *opacity_logit_out,
                             uint8_t *decayed, gsr_stream stream);

/* Camera poses around the renderer.  The renderer's d_pose is the gradient
 * w.r.t. a left perturbation T <- Exp(xi) T at the rendered pose (the
 * gradient of Eq. 11, se(3) ordered (rho, phi)).  These calls build the
 * cameras from two parameterisations and chain that gradient to them; one
 * thread per view, FP64 inside, asynchronous; no plan needed.  DEVICE arrays;
 * cams_out may alias cams_in.
 *
 * gsr_pose_apply: cams_out[v] = cams_in[v] with the pose Exp(xi_v) T_v, T_v
 * the pose (R, t) of cams_in[v], xi [n_views][6] = (rho, phi); Exp is the
 * SE(3) exponential [[R(phi), V(phi) rho], [0, 1]] (Rodrigues' formula).
 * gsr_pose_xi_grad: d_xi = J_l(xi)^T d_pose (written, [n_views][6]), the
 * gradient in xi of a loss of Exp(xi) T0 whose left-perturbation gradient at
 * Exp(xi) T0 is d_pose; J_l is the SE(3) left Jacobian. */
gsr_status gsr_pose_apply(gsr_ctx *ctx, int n_views, const float *xi, const gsr_camera *cams_in,
                          gsr_camera *cams_out, gsr_stream stream);
gsr_status gsr_pose_xi_grad(gsr_ctx *ctx, int n_views, const float *xi, const float *d_pose, float *d_xi,
                            gsr_stream stream);

/* The paper's pose parameters (supplement Sec. A: a quaternion q and a
 * translation t per pose, R from eq. q2R).  gsr_pose_from_qt: cams_out[v] =
 * cams_in[v] (intrinsics and size) with R = R(q_v / |q_v|), t = t_v; q
 * [n_views][4] = (q_r, q_i, q_j, q_k), nonzero; t [n_views][3].
 * gsr_pose_qt_grad: the gradient in (q, t) of a loss whose left-perturbation
 * gradient at [R(q/|q|) | t] is d_pose: d_t = d_pose[0:3] (moving t is the
 * translation perturbation) and d_q = (I - qh qh^T) / |q| times
 * (vee(dR/dqh_k R^T) . (g_phi + g_rho x t))_k -- the rotation that a change
 * of q makes, with the translation held (written; d_q [n_views][4], d_t
 * [n_views][3]).  With d_pose from GSR_PAPER_POSE_APPROX this is the paper's
 * own gradient through the projected centres and depths only. */
gsr_status gsr_pose_from_qt(gsr_ctx *ctx, int n_views, const float *q, const float *t, const gsr_camera *cams_in,
                            gsr_camera *cams_out, gsr_stream stream);
gsr_status gsr_pose_qt_grad(gsr_ctx *ctx, int n_views, const float *q, const float *t, const float *d_pose,
                            float *d_q, float *d_t, gsr_stream stream);

/* Per-stage timing of calls on this context (HIP events recorded on the
 * call's stream around each stage; HIP-graph launches are not split). */
enum {
  GSR_STAGE_PREPROCESS = 0, /* projection, binning data, depth keys */
  GSR_STAGE_DEPTH_SORT,     /* radix sort of the projected Gaussians by depth */
  GSR_STAGE_EMIT,           /* scan of tile counts and pair emission */
  GSR_STAGE_PAIR_SORT,      /* radix sort of the pairs by tile */
  GSR_STAGE_RANGES,         /* per-tile ranges and work order */
  GSR_STAGE_RASTER,         /* forward compositing, or the fused forward + L1 + backward */
  GSR_STAGE_RASTER_BWD,     /* backward compositing (unfused backward only) */
  GSR_STAGE_PREGRAD,        /* chain to parameters and pose */
  GSR_NSTAGES
};
/* Enable (1) or disable (0) stage timing for later calls. */
gsr_status gsr_set_profiling(gsr_ctx *ctx, int enable);
/* Synchronise, then return the summed milliseconds per stage (ms[GSR_NSTAGES])
 * and the number of timed calls since the last query; resets the sums. */
gsr_status gsr_stage_times(gsr_ctx *ctx, double *ms, int64_t *calls);

/* Work done by the last forward or fused call on `workspace` (synchronises
 * `stream`): out[0] = (tile, Gaussian) pairs, out[1] = pixel-Gaussian
 * evaluations of the forward walk (every list entry a pixel examined, up to
 * and including the one that stopped it), out[2] = entries blended,
 * out[3] = list entries the backward walk examines (sum of `last`).  The
 * render kernels do not count: this call walks the lists of that call again
 * with counting on, so `g` and `cfg` must be the ones that call used, with
 * their buffers unchanged.  Not on the hot path. */
gsr_status gsr_work_counts(gsr_ctx *ctx, const gsr_gaussians *g, const gsr_config *cfg, void *workspace,
                           gsr_stream stream, int64_t *out);

#ifdef __cplusplus
}
#endif
#endif /* GSR_H */
