/*
 * fmb.h -- C ABI of the MI355X (gfx950) sort-free Fuzzy Metaballs ray renderer.
 *
 * The renderer is the simplified two-parameter model of Keselman & Hebert,
 * "Flexible Techniques for Differentiable Rendering with 3D Gaussians" (WACV 2024):
 * every pixel ray meets every Gaussian at its peak density (Sec. 3.1, Eq. 2), the
 * per-Gaussian depths and normals (Eq. 17) are blended without sorting by the
 * two-parameter weights (Eq. 3 with Eq. 7), opacity follows Eq. (8), and per-pixel
 * optical flow is the change of the blended point's projection between two camera
 * poses (Sec. 5).  The backward pass returns the exact gradients of those outputs.
 *
 * Conventions shared by every call
 *   Gaussian i   mean mu_i (3 floats); precision Sigma_i^-1 = U_i^T U_i with U_i upper
 *                triangular, packed as (U00, U01, U02, U11, U12, U22) -- the paper's
 *                "inverse root precision" (Sec. 3.1); weight lambda_i > 0, linear (the
 *                kernels use log lambda_i, Eq. 2).
 *   blend        betas = (beta1, beta2) of Eq. (7), on the device (they are
 *                differentiated); eta > 0 is the shape scale of Eq. (7), a host value.
 *   colour       optional per-Gaussian colours [n,3], unconstrained; the rendered colour
 *                is sigmoid(q) per channel blended by Eq. (3) (Sec. 4: linear RGB).
 *   camera k     world-to-camera [R|T], row-major 3x4 (x_cam = R x_world + T), OpenCV
 *                axes (x right, y down, z forward); intrinsics (fx, fy, cx, cy); image
 *                H x W.  Pixel (row i, col j) has its centre at (j + 1/2, i + 1/2); its ray
 *                starts at the camera centre and has unit direction R^T d / |d| with
 *                d = ((j + 1/2 - cx)/fx, (i + 1/2 - cy)/fy, 1) (Sec. 5 camera model).
 *   rays         ordered view-major, then row-major: ray index of (k, i, j) is
 *                sum_{k'<k} H_k' W_k' + i W_k + j.  P is the total ray count.
 *   outputs      depth[P] = blended peak distance t_f along the unit ray (Eq. 3);
 *                alpha[P] (Eq. 8); normal[P,3] unit world-frame blended normal;
 *                flow[P,2] = pi_B(p) - pi_A(p) in pixels, p = origin + t_f * direction
 *                ([P,4] with a second flow target, see fmb_set_flow_pose2);
 *                color[P,3] blended colour; stash[P,8] = per-ray state the backward pass
 *                reads: (running max of the base-2 log weights, 1/sum of the shifted weights
 *                = max_i of the normalised weights (the Sec. 6 quality test), unnormalised
 *                blended normal (3), sum of densities, 0, 0).
 *
 * Memory: every float/int pointer called "device" is HIP device memory owned by the
 * caller; the library never frees it and reads/writes it only inside the calls.
 * "host" pointers are read during the call only.  All buffers are dense, row-major
 * and 4-byte aligned (16-byte aligned for stash).  All work is enqueued on the HIP
 * stream given (NULL = the default stream) and is asynchronous: results are ready
 * once that stream has been synchronised.
 *
 * Errors: every call returns FMB_OK (0) or a positive FMB_ERR_* code, never throws,
 * and leaves a thread-local message for fmb_last_error().  Argument checks happen
 * before any work is enqueued; a failed call enqueues nothing.
 */
#ifndef FMB_H
#define FMB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FMB_ABI_VERSION 3

/* Size limits, checked on the host before any work is enqueued (FMB_ERR_SHAPE beyond them):
 * rays of a scene, batch or loss call (2^31 - 2^24: every ray index and every tile end stays a
 * 32-bit int; per-ray output offsets such as 3 r or 4 r are formed in 64 bits), Gaussians of a
 * scene or batch, and views of a scene or batch. */
#define FMB_MAX_RAYS 2130706432LL
#define FMB_MAX_GAUSSIANS 268435455
#define FMB_MAX_VIEWS 134217727

enum fmb_status {
    FMB_OK = 0,
    FMB_ERR_INVALID_ARG = 1, /* null pointer, non-positive size, bad flag or value */
    FMB_ERR_SHAPE = 2,       /* sizes inconsistent with the scene or cameras */
    FMB_ERR_HIP = 3,         /* a HIP runtime call failed (message has hipGetErrorString) */
    FMB_ERR_OOM = 4,         /* device workspace allocation failed */
    FMB_ERR_CAPTURE = 5,     /* graph capture misuse (e.g. stream already capturing) */
    FMB_ERR_STATE = 6        /* call order violated (e.g. render before set_cameras) */
};

/* Blend weights of Eq. (3) (see fmb_set_model). */
enum fmb_model {
    FMB_MODEL_BLEND = 0,     /* two-parameter model: w_i = exp(beta1 d_i - beta2 t_i / eta) (Eq. 7) */
    FMB_MODEL_COMPOSITE = 1  /* zero-parameter model: alpha compositing (Eq. 9-10) */
};

typedef struct fmb_scene fmb_scene;
typedef struct fmb_batch fmb_batch;

/* ABI version of the loaded library (FMB_ABI_VERSION at build time). */
int fmb_abi_version(void);

/* Message of the last failed call on this thread ("" if none).  The pointer stays
 * valid until the next fmb_* call on the same thread. */
const char *fmb_last_error(void);

/* ------------------------------------------------------------------------------ */
/* Single scene                                                                   */
/* ------------------------------------------------------------------------------ */

/* Create a scene of 1 <= n <= FMB_MAX_GAUSSIANS Gaussians (representation of Sec. 3.1).
 *   means   device [n,3]; prec device [n,6] packed upper U; weights device [n] (> 0);
 *   betas   device [2] (beta1, beta2 of Eq. 7); eta host scalar > 0 (Eq. 7).
 * The pointers are BORROWED: they must stay valid while the scene is used and may be
 * updated in place between calls (each render/backward reads their current values).
 * Errors: FMB_ERR_INVALID_ARG for n < 1, a NULL pointer, eta <= 0 or misaligned input;
 * FMB_ERR_SHAPE for n > FMB_MAX_GAUSSIANS; FMB_ERR_HIP / FMB_ERR_OOM if the small device
 * descriptors cannot be created.
 * Values are not inspected (use fmb_validate). */
int fmb_scene_create(fmb_scene **out, int32_t n, const float *means, const float *prec,
                     const float *weights, const float *betas, float eta);

/* Point an existing scene at other parameter buffers of the same size n. */
int fmb_scene_rebind(fmb_scene *scene, const float *means, const float *prec,
                     const float *weights, const float *betas);

/* Release the scene and its workspace.  NULL is accepted.  The caller must make sure
 * no work using the scene is still running (synchronise its streams first). */
int fmb_scene_destroy(fmb_scene *scene);

/* Set the 1 <= v <= FMB_MAX_VIEWS views the scene is rendered from (all poses passed to the renderer,
 * Sec. 5).  w2c device [v,3,4]; intr device [v,4] (fx, fy, cx, cy); hw host [v,2]
 * (H, W >= 1).  w2c_b / intr_b: device [v,3,4] / [v,4] second pose per view for the
 * flow output, or both NULL (no flow).  Borrowed like the scene parameters.  Sizes the
 * workspace (P = sum H W rays, at most FMB_MAX_RAYS).
 * Errors: FMB_ERR_INVALID_ARG (NULL, v < 1, H or W < 1, only one of w2c_b/intr_b),
 * FMB_ERR_SHAPE (P > FMB_MAX_RAYS or v > FMB_MAX_VIEWS), FMB_ERR_OOM / FMB_ERR_HIP. */
int fmb_set_cameras(fmb_scene *scene, int32_t v, const float *w2c, const float *intr,
                    const int32_t *hw, const float *w2c_b, const float *intr_b);

/* Set the views and an explicit minibatch of rays instead of full images (the random ray
 * minibatches across all frames of Sec. 4).  counts host [v]: rays of each view (>= 0,
 * at least one > 0); rays are ordered view-major, view k's rays contiguous.  dirs device
 * [P,3]: world-frame directions (normalised by the kernels; non-zero), borrowed; every ray
 * starts at its view's camera centre.  w2c, intr, w2c_b, intr_b as fmb_set_cameras (intr is
 * used for the flow projections).  fmb_render / fmb_backward then work on these P rays.
 * Errors: as fmb_set_cameras. */
int fmb_set_rays(fmb_scene *scene, int32_t v, const float *w2c, const float *intr,
                 const int32_t *counts, const float *dirs, const float *w2c_b,
                 const float *intr_b);

/* Number of rays P of the current cameras (0 before fmb_set_cameras). */
int64_t fmb_num_rays(const fmb_scene *scene);

/* Add (or with NULL remove) a second flow target per view, so that every ray gets both the
 * forward and the backward flow (Sec. 5: poses i+1 and i-1): w2c_c device [v,3,4], intr_c
 * device [v,4] (batch: concatenated views), borrowed.  The flow output and cotangent then
 * have 4 columns per ray: (flow to pose B, flow to pose C).  Needs the first target
 * (w2c_b) to be set; fmb_set_cameras / fmb_set_rays clear it. */
int fmb_set_flow_pose2(fmb_scene *scene, fmb_batch *batch, const float *w2c_c,
                       const float *intr_c);

/* Choose the blend weights of a scene or batch (exactly one non-NULL); the default is
 * FMB_MODEL_BLEND.  FMB_MODEL_COMPOSITE is the zero-parameter renderer of Sec. 3.3:
 * w_i = T_i (1 - exp(-delta_i)), T_i = exp(-sum_j delta_j [t_j < t_i]) (Eq. 9-10; Gaussians
 * at equal t_i do not attenuate one another; in a scene of n Gaussians the densities below
 * 2^sig, sig = min(-30, -36 - ceil(log2 n)), are left out of the sums over j, which together
 * move a sum by less than 2^-36, and pairs whose density is below 2^skip of the ray's largest
 * weight, skip = min(-40, -26 - ceil(log2 n)), are left out of the blend and of its adjoint
 * (which keeps those with a density of at least 2^skip)), blended by Eq. (3) for depth,
 * normals and colour, alpha by Eq. (8) over every density; betas and eta are not
 * used and their gradient is 0.  Every
 * other call keeps its meaning, arguments and outputs; the stash holds the same fields
 * (the running maximum is that of log2 w_i).  Captured graphs are dropped when the model
 * changes; fmb_autotune leaves a compositing job as it is (one launch configuration).
 * Scenes of any size: a ray's significant intersections are taken in depth windows of at most
 * 48 Gaussians per ray tile, one window after another.
 * Errors: FMB_ERR_INVALID_ARG (bad model). */
int fmb_set_model(fmb_scene *scene, fmb_batch *batch, int32_t model);

/* Set (or with NULL clear) the per-Gaussian colours of a scene or batch (exactly one
 * non-NULL): device [n,3] (batch: [sum n,3]) unconstrained parameters q, borrowed; the
 * kernels use sigmoid(q) (Sec. 4).  Needed for a colour output / cotangent. */
int fmb_set_colors(fmb_scene *scene, fmb_batch *batch, const float *colors);

/* Forward pass (Eq. 2, 4, 7, 3, 8, 17 and the flow of Sec. 5) for all P rays.
 *   depth, alpha: device [P] (required); normal: device [P,3] or NULL (not computed:
 *   the normal terms are skipped); flow: device [P,2] or NULL (must be NULL when the
 *   cameras have no second pose); color: device [P,3] or NULL (needs fmb_set_colors);
 *   stash: device [P,8], 16-byte aligned, required by fmb_backward (may be NULL if no
 *   backward pass follows).
 * Errors: FMB_ERR_STATE (no cameras), FMB_ERR_INVALID_ARG, FMB_ERR_HIP. */
int fmb_render(fmb_scene *scene, float *depth, float *alpha, float *normal, float *flow,
               float *color, float *stash, void *stream);

/* Backward (adjoint) pass: gradients of  sum_r  g_depth[r] depth[r] + g_alpha[r] alpha[r]
 * + g_normal[r].normal[r] + g_flow[r].flow[r] + g_color[r].color[r]  with respect to the
 * means, packed precision factors, weights, colours and (beta1, beta2).  The per-pair
 * terms are recomputed, never stored.  Cotangents are device arrays shaped like the
 * outputs; any may be NULL (zero).  depth, color and stash are the forward outputs for the
 * SAME parameter values (color only needed with g_color).  Gradients are device arrays
 * g_means [n,3], g_prec [n,6], g_weights [n], g_colors [n,3] (or NULL), g_betas [2],
 * overwritten (not accumulated).  The result is deterministic (fixed reduction order).
 * g_normal needs the normals to have been rendered (their unnormalised sum is read from
 * the stash).  Errors: FMB_ERR_STATE, FMB_ERR_INVALID_ARG, FMB_ERR_HIP. */
int fmb_backward(fmb_scene *scene, const float *g_depth, const float *g_alpha,
                 const float *g_normal, const float *g_flow, const float *g_color,
                 const float *depth, const float *color, const float *stash, float *g_means,
                 float *g_prec, float *g_weights, float *g_colors, float *g_betas, void *stream);

/* Bytes of the fixed device workspace of fmb_backward_noalloc (32 MiB per device). */
#define FMB_NOALLOC_SCRATCH_BYTES (32ULL << 20)

/* fmb_backward for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same arguments, kernels and results
 * (bit for bit), with no device allocation.  The work lists, partial gradients and reduction
 * stages live in a fixed array of FMB_NOALLOC_SCRATCH_BYTES that the library holds on each device
 * it runs on until the process ends; the work lists are copied into it from host memory on
 * `stream` at every call (the scene's work plan is built on the host once per configuration).
 * Every call on a device shares that array and leaves its contents behind: calls that overlap on
 * one device (other streams or threads) race, and the caller must serialise them.  The scene's
 * device must be the current device.  Errors: those of fmb_backward; FMB_ERR_SHAPE when the
 * scene's work needs more workspace than FMB_NOALLOC_SCRATCH_BYTES (the message gives the size;
 * fmb_backward has no such limit); FMB_ERR_STATE when another device is current. */
int fmb_backward_noalloc(fmb_scene *scene, const float *g_depth, const float *g_alpha,
                         const float *g_normal, const float *g_flow, const float *g_color,
                         const float *depth, const float *color, const float *stash, float *g_means,
                         float *g_prec, float *g_weights, float *g_colors, float *g_betas, void *stream);

/* ------------------------------------------------------------------------------ */
/* Batch of independent scenes (uneven Gaussian counts, view counts, resolutions) */
/* ------------------------------------------------------------------------------ */

/* Create a batch of s >= 1 scenes rendered together by persistent kernels.
 *   n_host   host [s]: Gaussians per scene (>= 1); their parameters are concatenated
 *            scene after scene in means [sum n,3], prec [sum n,6], weights [sum n]
 *            (device); betas device [s,2]; eta host [s] (> 0).
 *   v_host   host [s]: views per scene (>= 1); cameras concatenated in the same order:
 *            w2c device [sum v,3,4], intr device [sum v,4], hw host [sum v,2],
 *            w2c_b / intr_b device or both NULL.
 * Rays and outputs are concatenated scene after scene, each scene in the single-scene
 * ray order.  All device pointers are borrowed (see fmb_scene_create).  The batch's total
 * Gaussians, views and rays are limited by FMB_MAX_GAUSSIANS, FMB_MAX_VIEWS and FMB_MAX_RAYS.
 * Errors: as fmb_scene_create and fmb_set_cameras. */
int fmb_batch_create(fmb_batch **out, int32_t s, const int32_t *n_host, const int32_t *v_host,
                     const float *means, const float *prec, const float *weights,
                     const float *betas, const float *eta, const float *w2c, const float *intr,
                     const int32_t *hw, const float *w2c_b, const float *intr_b);

int fmb_batch_destroy(fmb_batch *batch);

/* Total rays of the batch and the offset of scene `i`'s first ray / Gaussian. */
int64_t fmb_batch_num_rays(const fmb_batch *batch);
int64_t fmb_batch_ray_offset(const fmb_batch *batch, int32_t i);
int64_t fmb_batch_gauss_offset(const fmb_batch *batch, int32_t i);

/* Forward / backward over the whole batch with one persistent kernel each (work items
 * of (scene, view, ray tile) pulled from a device queue, largest first).  Arguments as
 * fmb_render / fmb_backward with concatenated arrays; g_betas is [s,2]. */
int fmb_batch_forward(fmb_batch *batch, float *depth, float *alpha, float *normal, float *flow,
                      float *color, float *stash, void *stream);
/* fmb_batch_forward with the gradient of the reconstruction loss's depth and alpha terms
 * (Sec. 4: binary cross entropy of alpha, clamped to [1e-6, 1 - 1e-6], against the target
 * mask alpha_t, plus w_depth times the alpha_t-weighted L1 depth error against depth_t, both
 * averaged over the batch's rays) written in the same pass: g_depth and g_alpha [P] receive
 * exactly what fmb_loss_grad writes for them, from the outputs this call renders, and no
 * separate pass over the outputs is needed.  Targets are caller-owned device arrays [P]; the
 * loss value itself and flow or colour terms are left to fmb_loss_grad.  Errors:
 * FMB_ERR_INVALID_ARG for a NULL batch, target or cotangent pointer or a non-finite w_depth,
 * and those of fmb_batch_forward. */
int fmb_batch_forward_loss(fmb_batch *batch, float *depth, float *alpha, float *normal, float *flow,
                           float *color, float *stash, const float *depth_t, const float *alpha_t,
                           float w_depth, float *g_depth, float *g_alpha, void *stream);
int fmb_batch_backward(fmb_batch *batch, const float *g_depth, const float *g_alpha,
                       const float *g_normal, const float *g_flow, const float *g_color,
                       const float *depth, const float *color, const float *stash,
                       float *g_means, float *g_prec, float *g_weights, float *g_colors,
                       float *g_betas, void *stream);

/* Capture the batch's forward pass and its backward pass, with these buffers, into two
 * HIP graphs held by the batch (replacing earlier ones).  `stream` must be a non-default
 * stream that is not already capturing (FMB_ERR_CAPTURE).  The graphs read the borrowed
 * parameters, cameras and cotangent buffers at replay time, so in-place updates between
 * replays are seen (a loss can fill the cotangents between the two replays).
 * fmb_batch_graph_launch replays the forward (which = 0), the backward (1) or both (2)
 * on `stream`; FMB_ERR_STATE if nothing was captured.  Replays of one batch must not
 * overlap (they share the batch's work counters and partial-gradient workspace).
 * The graphs are dropped (the next fmb_batch_graph_launch returns FMB_ERR_STATE until the
 * batch is captured again) by every call that changes what they launch: fmb_autotune,
 * fmb_set_config, fmb_set_model, fmb_set_colors and fmb_set_flow_pose2 with a changed
 * value, and any eager forward or backward call that rebuilds the work lists (a backward
 * with a colour cotangent after one without, or the reverse).  Graphs that a caller
 * captures itself around library calls (e.g. one graph of a whole training step) hold
 * the same kernel arguments and workspace addresses: after any of these calls they must be
 * captured again; replaying them is undefined. */
int fmb_batch_capture(fmb_batch *batch, float *depth, float *alpha, float *normal, float *flow,
                      float *color, float *stash, const float *g_depth, const float *g_alpha,
                      const float *g_normal, const float *g_flow, const float *g_color,
                      float *g_means, float *g_prec, float *g_weights, float *g_colors,
                      float *g_betas, void *stream);
int fmb_batch_graph_launch(fmb_batch *batch, int32_t which, void *stream);

/* ------------------------------------------------------------------------------ */
/* Tuning and diagnostics                                                         */
/* ------------------------------------------------------------------------------ */

/* Time the compiled tile configurations of the forward and backward kernels on the
 * scene's (or batch's) current shapes and keep the fastest.  This runs real kernels on
 * `stream` with the given buffers (outputs and gradients are overwritten); the backward
 * variants are timed with the cotangents given (NULL ones stay NULL, as in the real
 * step).  If cache_path is non-NULL the choice is read from / appended to that text
 * file, keyed by device, kernel version, shapes and which outputs/cotangents are used.
 * Exactly one of `scene` and `batch` is non-NULL. */
int fmb_autotune(fmb_scene *scene, fmb_batch *batch, float *depth, float *alpha, float *normal,
                 float *flow, float *color, float *stash, const float *g_depth,
                 const float *g_alpha, const float *g_normal, const float *g_flow,
                 const float *g_color, float *g_means, float *g_prec, float *g_weights,
                 float *g_colors, float *g_betas, const char *cache_path, void *stream);

/* Gradient of the reconstruction loss of Sec. 4 (Eq. 11-14) with respect to one render's
 * outputs, averaged over its p rays (the cotangents fmb_backward takes):
 *   L = 1/p sum_r [ -(a*_r log a_r + (1 - a*_r) log(1 - a_r))      a_r = clamp(alpha_r,
 *                                                                   1e-6, 1 - 1e-6)  (Eq. 11)
 *                 + w_depth a*_r |depth_r - depth*_r|               (mask-weighted L1)
 *                 + w_color a*_r |color_r - color*_r|_1              (Eq. 12)
 *                 + w_flow  a*_r |flow_r - flow*_r|_q ]             (Eq. 13; q = 1: L1 of
 *                                                                   the flow components, q = 2:
 *                                                                   squared L2)
 * where a* = alpha_t is the target mask (the paper's lambda_C = 4.5 and lambda_F = 210 are
 * w_color and w_flow).  depth, alpha, depth_t, alpha_t: device [p]; flow, flow_t: device
 * [p,flow_cols] (flow_cols 2, or 4 for forward and backward flow) or NULL (no flow term;
 * then g_flow must be NULL too); color, color_t: [p,3] or NULL likewise.  g_depth, g_alpha:
 * device [p] (written); g_flow [p,flow_cols], g_color [p,3] or NULL.  The clamp passes the gradient where 1e-6 <= alpha <= 1 - 1e-6 (float32 bounds);
 * |x|' is sign(x) (0 at 0).  block_loss: device [ceil(p / 1024)] or NULL; if given,
 * receives per-block partial sums of L (sum them for the loss; the order is fixed).
 * Errors: FMB_ERR_INVALID_ARG (p < 1, NULL required pointer, flow_norm not 1 or 2,
 * flow_cols not 2 or 4), FMB_ERR_SHAPE (p > FMB_MAX_RAYS). */
int fmb_loss_grad(int64_t p, const float *depth, const float *alpha, const float *flow,
                  const float *color, const float *depth_t, const float *alpha_t,
                  const float *flow_t, const float *color_t, float w_depth, float w_flow,
                  int32_t flow_norm, int32_t flow_cols, float w_color, float *g_depth, float *g_alpha,
                  float *g_flow, float *g_color, float *block_loss, void *stream);

/* Split statistic of Sec. 8 for a scene or batch (exactly one non-NULL): the average loss
 * assigned to each Gaussian over the M rays of its scene,
 *   lbar_i = (1/M) sum_j loss_j w_ji,
 * w_ji the normalised Eq. (3) weights of the current model (Eq. 7 or Eq. 9-10).  loss: device
 * [P] per-ray loss (any reconstruction loss; typically over a random ~5 % of the rays set with
 * fmb_set_rays); stash: device [P,8] from the forward pass of the same model and parameters;
 * lbar: device [n] (batch: [sum n]), written.  Sums run in a fixed order (deterministic).
 * Errors: FMB_ERR_STATE (no cameras), FMB_ERR_INVALID_ARG, FMB_ERR_HIP. */
int fmb_split_statistic(fmb_scene *scene, fmb_batch *batch, const float *loss, const float *stash,
                        float *lbar, void *stream);

/* Removal and splitting of Gaussians (Sec. 8), host arrays, double-precision host code.
 *
 * fmb_prune_mask: remove[i] = 1 where weights[i] <= mean - z * std over the n weights (the
 * population standard deviation; the paper's z is 2), else 0.
 * fmb_split_mask: split[i] = 1 where lbar[i] >= mean + z * std over the n values (z = 1 in
 * the paper; lbar from fmb_split_statistic), else 0.
 * fmb_split_gaussians: each of the n given Gaussians becomes two, written at 2i and 2i + 1:
 * means mu +- sigma_1 sqrt(2/pi) v_1 (v_1 the dominant axis of Sigma, sigma_1 the standard
 * deviation along it, v_1's largest-magnitude component taken positive), both with Sigma's
 * axes and sigma_1 scaled by sqrt(1 - 2/pi) (packed upper factor of the new precision, positive
 * diagonal); weights lambda exp(noise_w[k]) and colours (unconstrained) colors + noise_c[k],
 * the noise drawn by the caller (the paper: N(0, 0.1^2) each).  means [n,3], prec [n,6],
 * weights [n], colors [n,3] or NULL, noise_w [2n], noise_c [2n,3] (NULL with colors NULL);
 * outputs out_means [2n,3], out_prec [2n,6], out_weights [2n], out_colors [2n,3] or NULL.
 * Errors: FMB_ERR_INVALID_ARG (bad sizes or pointers, a precision factor that is not
 * positive definite). */
int fmb_prune_mask(int32_t n, const float *weights, float z, uint8_t *remove);
int fmb_split_mask(int32_t n, const float *lbar, float z, uint8_t *split);
int fmb_split_gaussians(int32_t n, const float *means, const float *prec, const float *weights,
                        const float *colors, const float *noise_w, const float *noise_c,
                        float *out_means, float *out_prec, float *out_weights, float *out_colors);

/* Pin the launch configuration of a scene or batch (exactly one non-NULL) instead of
 * autotuning it: forward variant in [0, 4), backward variant in [0, 9) (see
 * fmb_get_config), persistent-grid multipliers 1 or 2.  Every variant computes the same
 * results to rounding; captured graphs are dropped.  Until this call or fmb_autotune, a job
 * takes forward variant 1 (512 rays per item), or 0 (256) when it has fewer rays than two
 * 512-ray items per compute unit, and backward variant 8 (variant 2 for calls with a normal or
 * colour cotangent).  Errors: FMB_ERR_INVALID_ARG. */
int fmb_set_config(fmb_scene *scene, fmb_batch *batch, int32_t fwd_variant, int32_t bwd_variant,
                   int32_t fwd_grid_mult, int32_t bwd_grid_mult);

/* Current launch configuration of a scene or batch (exactly one non-NULL), written to the
 * host array out[8]: forward tile variant, rays per forward work item, backward variant,
 * rays per backward tile (staged in LDS for variants 0-2, which give each lane a Gaussian;
 * held by the block's lanes for variants 3-5, which give each lane rays as the forward pass
 * does and sum each Gaussian's terms over the wave per tile; the rays of an item, 8 or 16 tiles
 * of 8 x 8 pixels, for variants 6-8 (8: blocks of 512 threads), which give each lane a ray of
 * a tile and each wave a Gaussian at a time -- they take no normal cotangent, and calls with
 * one run variant 2), forward and backward persistent-grid multipliers, and the
 * forward and backward work-item counts (0 until the first call built them). */
int fmb_get_config(const fmb_scene *scene, const fmb_batch *batch, int32_t *out);

/* Check the scene's parameters on the device: writes to *bad_host a bit mask of
 * 1 = non-finite value, 2 = weight <= 0, 4 = zero diagonal entry of U, 8 = beta not
 * finite, and synchronises `stream`. */
int fmb_validate(fmb_scene *scene, int32_t *bad_host, void *stream);

/* Kernel timing: when enabled, each fmb_render / fmb_backward / fmb_batch_* call
 * records HIP events around its main kernels on the call's stream (around the whole
 * graph for fmb_batch_graph_launch; nothing while a stream is capturing), and
 * fmb_kernel_times returns the summed milliseconds and launch counts
 * (fwd_ms, bwd_ms, fin_ms, n_fwd, n_bwd, n_fin) since the last reset. */
int fmb_timing_enable(int enable);
int fmb_kernel_times(double *out6, int reset);

#ifdef __cplusplus
}
#endif

#endif /* FMB_H */
