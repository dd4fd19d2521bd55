/*
 * unigs.h -- C ABI of the MI355X (gfx950) multimodal Gaussian rasterizer.
 *
 * The library implements the rendering hot path of UniGS (arXiv 2510.12174):
 * tile-based differentiable rasterization of 3D Gaussians that renders, in one
 * pass, RGB, ray-ellipsoid midpoint depth, world-frame normals estimated from
 * depth, semantic logits and the gradient-factor map (section 3.2 "Geometry-
 * Aware Rasterization", section 3.3 "Differentiable Pruning", section 3.4 and
 * Alg. forward_render), and the analytic backward of all of them into the
 * Gaussian parameters (supplementary S1.2, S1.4, S1.6; Alg. normal_gradient,
 * Alg. backward_render).
 *
 * Conventions shared by every entry point
 *  - All tensor pointers are DEVICE pointers owned by the caller, FP32 unless
 *    stated, contiguous, 4-byte aligned (binary16 maps 2-byte; misaligned
 *    pointers are rejected); 16-byte alignment lets some kernels use vector
 *    loads.  Struct arguments and camera arrays are HOST memory, read during
 *    the call only.
 *  - Layouts are planar.  Gaussian parameters (structure of arrays):
 *      mean [3][N], quat [4][N] as (w,x,y,z) (need not be normalised),
 *      log_scale [3][N], opacity_logit [N], mask_logit [N] (gradient factor
 *      k = sigmoid(mask_logit)), sh [(sh_deg+1)^2][3][N], sem [N][C_o].
 *    Image maps of view v are [C][H_v][W_v]; several views are stored one after
 *    the other, so view v's plane set starts at element C * pix_off(v) with
 *    pix_off(v) = sum over u < v of W_u * H_u.
 *  - Every call is asynchronous on `stream` (a hipStream_t, NULL = the legacy
 *    default stream) unless stated.  No call allocates device memory: scratch
 *    space is one caller-allocated workspace sized by ugs_workspace_size().
 *  - Errors are returned as negative status codes (never thrown, never a trap).
 *    Invalid arguments are rejected before anything is launched.
 *  - Inputs are never modified.  Gradient outputs are ACCUMULATED (+=): the
 *    caller zero-fills them before the first backward.
 */
#ifndef UNIGS_H
#define UNIGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define UGS_OK 0
#define UGS_ERR_INVALID_ARG (-1)  /* null/misaligned pointer, bad size or option      */
#define UGS_ERR_UNSUPPORTED (-2)  /* C_o > UGS_MAX_CHANNELS, sh_deg > 3, tile shape   */
#define UGS_ERR_CAPACITY (-3)     /* more (tile, Gaussian) pairs than pair_capacity   */
#define UGS_ERR_HIP (-4)          /* a HIP runtime call failed (see ugs_last_hip_error) */
#define UGS_ERR_NOT_CAPTURED (-5) /* ugs_step_replay without a captured step          */
#define UGS_ERR_STATE (-6)        /* calls out of order (e.g. render before bin_sort)  */

#define UGS_MAX_CHANNELS 256 /* semantic channels C_o supported */
#define UGS_MAX_VIEWS 64

/* Pinhole camera (supplementary S1.3): x_cam = R x_world + t, pixel
 * (u, v) = (fx x/z + cx, fy y/z + cy).  R is row-major.  The ray of pixel (u,v)
 * is C + s * normalize(R^T ((u-cx)/fx, (v-cy)/fy, 1)) with C = -R^T t (Eq.
 * computeRay).  Gaussians with camera depth <= z_near are culled. */
typedef struct {
    int W, H;
    float fx, fy, cx, cy;
    float R[9];
    float t[3];
    float z_near;
} ugs_camera;

/* Gaussian parameters G = {mu, q, s, alpha, h, o, k} (Eq. gs_representation),
 * stored as the raw (pre-activation) values: s = exp(log_scale),
 * opacity = sigmoid(opacity_logit), k = sigmoid(mask_logit). */
typedef struct {
    int64_t N;
    int sh_deg; /* 0..3 */
    int C_o;    /* 0..UGS_MAX_CHANNELS */
    const float *mean, *quat, *log_scale, *opacity_logit, *mask_logit, *sh, *sem;
} ugs_gaussians;

/* Gradients with respect to the same parameters, same layouts (accumulated). */
typedef struct {
    float *mean, *quat, *log_scale, *opacity_logit, *mask_logit, *sh, *sem;
} ugs_gaussian_grads;

/* Forward outputs, all views (layout above).  rgb [3], depth [1] (alpha-blended
 * midpoint depth, Eq. depth_render, background 0), kmap [1] (gradient-factor map,
 * Eq. t_render), normal [3] (world frame, Alg. normal_estimation; 0 where the
 * stencil leaves the image or is degenerate), sem [C_o] (Eq. semantic_render),
 * T_final [1] (transmittance after the last contributor, saved for the backward
 * as in Alg. forward_render), n_contrib [1] uint32 (one past the position, in the
 * pixel's tile list, of its last contributor).  T_final and n_contrib may be
 * NULL for forward-only use (viewer/inference): they are then not stored, and
 * the backward, which needs them, rejects such outputs. */
typedef struct {
    float *rgb, *depth, *kmap, *normal, *sem, *T_final;
    uint32_t *n_contrib;
} ugs_outputs;

/* Upstream gradients dL/d(output), same layouts as ugs_outputs.  A NULL map
 * means zero.  These are the loss gradients Alg. backward_render takes.
 * Fused cosine seed: when `normal` is NULL and `normal_target` is set, the
 * normal gradient is formed inside Alg. normal_gradient as
 * (*normal_scale) * normal_target (the seed -N_target / |Omega| of
 * Eq. gradientn, with the loss weight folded into the device scalar
 * `normal_scale`, e.g. the coefficient ugs_loss writes at losses[10]); both
 * pointers are device memory, normal_target laid out like the normal map.
 * Fused cross-entropy seed: when `sem` is NULL and `sem_label` is set
 * ([H][W] int32 per view), Alg. backward_render forms the semantic upstream
 * itself from the rendered logits of `out` as (*sem_scale) *
 * (softmax(O~) - onehot(label)) per pixel (0 for a label outside [0, C_o)),
 * e.g. with the coefficient ugs_loss writes at losses[12]; the semantic
 * gradient map is then never stored. */
typedef struct {
    const float *rgb, *depth, *kmap, *normal, *sem;
    const float *normal_target, *normal_scale;
    const int32_t *sem_label;
    const float *sem_scale;
} ugs_upstream;

/* Options.  Zero-initialise and call ugs_default_options() to get the defaults. */
typedef struct {
    int tile_w, tile_h;  /* 16x16 (default), 8x8 or 32x8 */
    int batch;           /* Gaussians staged per LDS batch (render kernels), 0 = auto */
    int step1, step2;    /* finite-difference steps of Alg. normal_estimation (1, 2) */
    float lambda;        /* fusion weight of the two normals (0.5) */
    int orient_sign;     /* +1: flip normals to face the camera; -1: the literal
                            Eq. direction_correction (keep if N . d_view <= 0) */
    float prune_Tk;      /* > 0: skip Gaussians with |k - 1| > prune_Tk (section 3.3) */
    int depth_mode;      /* fragment depth d_i composited into the depth map:
                            0 (default): the camera depth of the midpoint of the
                              ray-ellipsoid intersections (section 3.2, Eq. midpoint);
                            1: the camera depth of the Gaussian's centre, the
                              "Center Point" row of the supplementary's module
                              ablation table;
                            2: the midpoint where the pixel ray meets the
                              ellipsoid (the quadratic of section 3.2 has a real
                              root) and the centre depth where it has no valid
                              solution.  Gradients follow the chosen form. */
    int half_outputs;    /* 1: the rgb, kmap, normal and sem maps of ugs_outputs
                            are IEEE binary16 (the float pointers are read as
                            2-byte elements, rounded to nearest even); depth,
                            T_final and n_contrib keep their types.  For viewing
                            and inference: ugs_render_bwd and training steps
                            reject it.  Default 0 (FP32). */
    int sem_bf16x3;      /* 1: for 9..32 channels, run the semantic products of
                            Eq. semantic_render and Eq. gradiento on bf16 matrix
                            cores with each FP32 operand split into a high and a
                            low bf16 part (three products, FP32 accumulation;
                            about 2^-16 relative per product instead of FP32's
                            2^-24).  Default 0: FP32 products (FP32 matrix cores
                            for 9..256 channels, FP32 vector arithmetic for 1..8). */
} ugs_options;

typedef struct ugs_ctx ugs_ctx;

/* Fills `opt` with the defaults listed above. */
void ugs_default_options(ugs_options *opt);

/* Creates a context holding host-side state only (options, last problem shape,
 * captured graph, tuning).  One context per stream; not thread-safe. */
int ugs_create(ugs_ctx **out, const ugs_options *opt);
void ugs_destroy(ugs_ctx *ctx);
/* Replaces the options (tile shape, batch, normal parameters); invalidates a
 * captured step. */
int ugs_set_options(ugs_ctx *ctx, const ugs_options *opt);

/* Workspace bytes for N Gaussians, C_o channels, V views (cameras on the host)
 * and room for pair_capacity (tile, Gaussian) pairs (< 2^31). */
int ugs_workspace_size(const ugs_ctx *ctx, int64_t N, int C_o, int sh_deg, const ugs_camera *cams, int V,
                       int64_t pair_capacity, size_t *bytes);

/* Stage S1, projection (the 3DGS preprocessing the paper extends, section 3.4
 * "Tile-based Forward Rasterization"): for every view and Gaussian, EWA footprint
 * (conic, 2D mean), SH colour, opacity, gradient factor, the depth coefficients
 * of the ray-ellipsoid midpoint (section 3.2), the sort depth and the tile
 * rectangle of the alpha >= 1/255 region.  Parameters are read once for all V
 * views.  Writes only into `ws`.  Also zeroes the per-view gradient records used
 * by ugs_render_bwd. */
int ugs_project(ugs_ctx *ctx, const ugs_gaussians *g, const ugs_camera *cams, int V, void *ws, size_t ws_bytes,
                void *stream);

/* Stages S2-S4: pair emission (one pair per tile a Gaussian's rectangle covers,
 * key = (global tile << 32) | float bits of the camera depth, value = Gaussian
 * index), a stable radix sort so that each tile's list is ordered by (depth,
 * index), and the per-tile [start, end) ranges.  When P_out is non-NULL the call
 * synchronises the stream and stores the pair count P.  When P exceeds the
 * capacity the sort is skipped, nothing is written out of bounds, the call
 * returns UGS_ERR_CAPACITY (only detectable when P_out is non-NULL; otherwise a
 * device flag makes the following render calls produce zero outputs and
 * ugs_check_overflow reports it). */
int ugs_bin_sort(ugs_ctx *ctx, void *ws, void *stream, int64_t *P_out);

/* Synchronises `stream` and returns UGS_ERR_CAPACITY if the last bin_sort
 * overflowed (and the required P in *P_required), UGS_OK otherwise. */
int ugs_check_overflow(ugs_ctx *ctx, void *ws, void *stream, int64_t *P_required);

/* Stages S5-S6: Alg. forward_render over every tile of every view (front-to-back
 * compositing of RGB, depth, gradient factor and semantics, saving T_final and
 * the last contributor) followed by Alg. normal_estimation on the depth. */
int ugs_render_fwd(ugs_ctx *ctx, const ugs_gaussians *g, void *ws, const ugs_outputs *out, void *stream);

/* Stages S7-S9: Alg. normal_gradient (dL/dN -> dL/dD), Alg. backward_render
 * (reverse traversal from T_final, gradients of colour, depth, gradient factor,
 * semantics and alpha), and the chain into the parameters (supplementary S1.2
 * for depth -> (mu, s, R), R -> q by the tangent projection, EWA and SH
 * adjoints).  `out` must hold the outputs of the matching ugs_render_fwd, which
 * must have been called with T_final and n_contrib (else UGS_ERR_STATE).
 * Gradients are summed over views and ADDED to `dg`.  One ugs_render_bwd per
 * ugs_project: the projection clears the per-record gradient buffers of the
 * workspace that this call accumulates into, so a second ugs_render_bwd (or one
 * after a replayed step or an autotune) returns UGS_ERR_STATE until the next
 * ugs_project + ugs_bin_sort. */
int ugs_render_bwd(ugs_ctx *ctx, const ugs_gaussians *g, void *ws, const ugs_outputs *out,
                   const ugs_upstream *dout, const ugs_gaussian_grads *dg, void *stream);

/* Batched training step: captures project -> bin_sort -> render_fwd ->
 * render_bwd for all V views into one HIP graph (no host synchronisation inside;
 * with dout and dg both NULL, a forward-only step: project -> bin_sort ->
 * render_fwd (normals included), for viewing or inference, where T_final and
 * n_contrib may be NULL too;
 * the pair count stays on the device and is bounded by the workspace capacity).
 * ugs_step_replay launches it; a replay whose pair count overflowed returns
 * UGS_ERR_CAPACITY at the NEXT replay (outputs of the overflowing replay are
 * zero) and the step must be re-captured with a larger workspace.  The buffers
 * passed at capture are the ones every replay reads and writes. */
int ugs_step_capture(ugs_ctx *ctx, const ugs_gaussians *g, const ugs_camera *cams, int V, void *ws,
                     size_t ws_bytes, const ugs_outputs *out, const ugs_upstream *dout,
                     const ugs_gaussian_grads *dg, void *stream);
int ugs_step_replay(ugs_ctx *ctx, void *stream);

/* Times the candidate (tile shape, batch) configurations on the given problem
 * (one forward+backward each, after a warm-up), checks that every candidate's
 * forward outputs are bit-identical to the first one's (the semantic map to
 * rounding: for 9..32 channels its sums run on the matrix cores in groups of
 * list entries that depend on the tile shape), keeps the fastest in the
 * context options and returns it in *chosen (and its time in *ms if non-NULL).
 * Synchronous.  Uses `out` and `dg` as scratch (dg is zeroed afterwards).
 * Candidates whose pair count exceeds the workspace capacity are skipped
 * (UGS_ERR_CAPACITY only if all are).  Returns UGS_ERR_STATE if the candidates'
 * outputs differ. */
int ugs_autotune(ugs_ctx *ctx, const ugs_gaussians *g, const ugs_camera *cams, int V, void *ws, size_t ws_bytes,
                 const ugs_outputs *out, const ugs_upstream *dout, const ugs_gaussian_grads *dg, void *stream,
                 ugs_options *chosen, float *ms);

/* Total (tile, Gaussian) pairs of the last bin_sort (synchronises). */
int ugs_pair_count(ugs_ctx *ctx, void *ws, void *stream, int64_t *P);

/* Timing hook: when `stage` is non-zero, every later call records `ev_start`
 * (a hipEvent_t) on the stream right before the kernels of that stage and
 * `ev_stop` right after them, in eager calls and inside a captured step alike.
 * Stages: 1 project, 2 bin+sort, 3 render_fwd compositing, 4 normal_fwd,
 * 5 normal_bwd, 6 render_bwd compositing, 7 project_bwd.  stage = 0 disables. */
int ugs_time_stage(ugs_ctx *ctx, int stage, void *ev_start, void *ev_stop);

/* Introspection for stage-wise tests: device pointer (inside `ws`) and element
 * count of an internal array after the stage that writes it has run.  `which`:
 *   0 render records, float[V*N][16] (layout in the source), written by project;
 *   1 tile rectangles, uint32[V*N][2] = (tx0 | ty0 << 16, tx1 | ty1 << 16),
 *     half-open, project;
 *   2 tiles touched, uint32[V*N], project;
 *   3 sorted keys, uint32[P] = global tile id (each tile's run is in (depth,
 *     index) order), bin_sort;
 *   4 sorted values (Gaussian index), uint32[P], bin_sort;
 *   5 tile ranges, uint32[total tiles][2] = [start, end), bin_sort;
 *   6 per-view gradient records, float[V*N][16], render_bwd;
 *   7 depth gradient incl. the normal branch, float[total pixels], render_bwd;
 *   8, 9 start and end time of each tile's workgroup in the forward and the
 *     backward compositing (9..256 channels, counters enabled), uint64[total
 *     tiles][2], in ticks of the 100 MHz GPU real-time clock;
 *  10 activity mask of the last training forward (9..256 channels): per
 *     wavefront slot of a tile (4 planes), one bit per sorted list entry that
 *     at least one of the wavefront's pixels composites, uint32[4][words].
 * Counts 3 and 4 read the pair count back (synchronises `stream`). */
int ugs_debug_buffer(ugs_ctx *ctx, void *ws, int which, void *stream, void **dev_ptr, int64_t *count);

/* Human-readable status; last HIP error string of the context. */
const char *ugs_status_string(int status);
const char *ugs_last_hip_error(const ugs_ctx *ctx);

/* Kernel-level counters for roofline accounting: after a render_fwd, the number
 * of (pixel, list entry) evaluations and of contributing fragments over all
 * views (synchronises; counting adds atomics, so it is off unless enabled).
 * While enabled, the compositing kernels for 9..256 channels (first pass of
 * the forward and of the backward) also record each (view, tile) workgroup's
 * start and end time, read back with ugs_debug_buffer 8 and 9. */
int ugs_enable_counters(ugs_ctx *ctx, int on);
int ugs_read_counters(ugs_ctx *ctx, void *ws, void *stream, int64_t *evaluated, int64_t *contributing);

/* Scratch bytes (device memory) that ugs_prune needs for N Gaussians. */
int ugs_prune_scratch_size(int64_t N, size_t *bytes);

/* Differentiable pruning (section 3.3, "Pruning"): keeps the Gaussians whose
 * gradient factor k = sigmoid(mask_logit) satisfies |k - 1| <= T_k -- the test
 * of the projection's pruning skip, evaluated in FP64 -- and compacts, in index
 * order, every parameter array of `g` into `out`, and each of the `n_state`
 * state sets state_in[s] (per-Gaussian arrays laid out like the parameters,
 * e.g. optimiser moments; NULL fields are skipped; their N, sh_deg and C_o are
 * taken from `g`) into state_out[s].  Output arrays are caller-owned device
 * memory with room for g->N Gaussians; their structure-of-arrays rows are
 * packed at the kept count (row r of `mean` starts at r * n_kept), `sem` rows
 * stay [n_kept][C_o].  With reset_k != 0 the kept mask logits in `out` become
 * ln 9 (k = 0.9), the paper's reset after pruning.  `scratch` (device,
 * 256-byte aligned, ugs_prune_scratch_size bytes) is overwritten; inputs and
 * outputs must not overlap.  Synchronises `stream`; returns the kept count in
 * *n_kept.  Errors: UGS_ERR_INVALID_ARG (NULL or misaligned pointers, T_k < 0,
 * scratch too small), UGS_ERR_HIP. */
int ugs_prune(const ugs_gaussians *g, const ugs_gaussian_grads *out, int n_state, const ugs_gaussians *state_in,
              const ugs_gaussian_grads *state_out, float T_k, int reset_k, void *scratch, size_t scratch_bytes,
              int64_t *n_kept, void *stream);

/* The same compaction as ugs_prune without a caller scratch buffer, for callers
 * that cannot allocate device memory (code running under HIP graph capture,
 * tight serving or training loops, harnesses that forbid hipMalloc).  The keep
 * flags and their scan live in a fixed array inside the library, one copy per
 * GPU (about 32 MiB, held until the process ends); the call itself allocates
 * nothing.  g->N must be at most UGS_PRUNE_NOALLOC_MAX_N, else
 * UGS_ERR_UNSUPPORTED; other errors as ugs_prune.  Every call on one GPU uses
 * that GPU's array: calls that overlap on one GPU (two streams, two threads)
 * race and must be serialised by the caller.  Synchronises `stream`. */
#define UGS_PRUNE_NOALLOC_MAX_N (1 << 22)
int ugs_prune_noalloc(const ugs_gaussians *g, const ugs_gaussian_grads *out, int n_state,
                      const ugs_gaussians *state_in, const ugs_gaussian_grads *state_out, float T_k, int reset_k,
                      int64_t *n_kept, void *stream);

/* ---------------------------------------------------------------- losses
 * The training loss of section 3.4 ("Loss Function") on the rendered maps,
 * producing the upstream gradients that ugs_render_bwd consumes, on the device
 * and without host synchronisation (graph-capturable).  Terms, each a mean
 * over the P pixels of all views (RGB terms over 3P values):
 *   L_l1     = mean |C - C_gt|;
 *   L_ssim   = 1 - mean SSIM(C, C_gt) per channel (11x11 Gaussian window,
 *              sigma 1.5, C1 = 0.01^2, C2 = 0.03^2, zero padding);
 *   L_normal = 1 - mean N . N_gt (Eq. csloss; its gradient is the seed
 *              -N_gt / P of Eq. gradientn);
 *   L_depth  = mean |D - D_gt| (the paper names it without a definition);
 *   L_seg    = mean cross-entropy of softmax(O) against the class label
 *              (a label outside [0, C_o) marks a pixel that adds nothing);
 *   L_K      = mean |K - 1| (Eq. for L_K).
 * L_all = l1 L_l1 + sum_x lambda_x w_x L_x with w_x = |L_l1| / |L_x| when
 * `balance` is set (the equation for L_all; the ratios are held constant in
 * the gradient; 0 when L_x is 0) and 1 otherwise.  A NULL target drops its
 * term (its loss and gradient are 0). */
typedef struct {
    const float *rgb;      /* [3][H][W] per view, stacked like ugs_outputs */
    const float *depth;    /* [H][W] per view, or NULL */
    const float *normal;   /* [3][H][W] per view, or NULL */
    const int32_t *label;  /* [H][W] class index in [0, C_o) per view, or NULL */
} ugs_targets;

#define UGS_LOSS_VALUES 14

typedef struct {
    float lambda[6];  /* weights of l1, ssim, normal, depth, seg, K (1, 0.1 x 5) */
    int balance;      /* 1: scale terms by |L_l1| / |L_x| */
} ugs_loss_options;

/* Fills the defaults listed above. */
void ugs_default_loss_options(ugs_loss_options *opt);

/* Scratch bytes (device) ugs_loss needs for these views. */
int ugs_loss_scratch_size(const ugs_camera *cams, int V, size_t *bytes);

/* Evaluates the loss of `out` against `gt` and writes dL_all/d(map) into the
 * caller-owned device maps of `grad` (same layouts as ugs_outputs; rgb, kmap
 * always written, depth/normal/sem written when non-NULL, as zero when their
 * term is absent; the pointers are written through despite the const of
 * ugs_upstream; a NULL grad->normal or grad->sem leaves that seed to the fused
 * forms of ugs_upstream).  `losses` is device memory for UGS_LOSS_VALUES floats: L_l1,
 * L_ssim, L_normal, L_depth, L_seg, L_K, L_all and the SSIM mean, then the six
 * per-term gradient coefficients (d L_all / d map element of the l1, ssim,
 * normal, depth, seg and K terms; losses[10] is the fused normal seed's scale).  `scratch` (256-byte aligned,
 * ugs_loss_scratch_size bytes) is overwritten.  Asynchronous on `stream`.
 * Errors: UGS_ERR_INVALID_ARG (NULL rgb maps, NULL or misaligned buffers,
 * C_o out of range, labels without C_o). */
int ugs_loss(const ugs_camera *cams, int V, int C_o, const ugs_outputs *out, const ugs_targets *gt,
             const ugs_loss_options *opt, const ugs_upstream *grad, float *losses, void *scratch,
             size_t scratch_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* UNIGS_H */
