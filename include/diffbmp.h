/*
 * diffbmp.h -- C ABI of the MI355X (gfx950) differentiable bitmap-primitive rasteriser.
 *
 * The operation is DiffBMP's renderer (arXiv 2602.22625, Sec. 3.1): N bitmap primitives, each
 * with position (x, y), scale s, rotation theta, opacity logit nu and colour logits c in R^3,
 * are mapped onto an H x W canvas by the inverse affine map of Eq. (1), sampled bilinearly at
 * the bitmap coordinates of Eq. (2) (Supp. Eqs. S1-S3), given opacity
 *     alpha_k = alpha_max * sigmoid(nu_k) * M_k(x, y)                         (Eq. 3)
 * and composited front to back with Porter-Duff over (Eqs. 4-5), index 0 in front:
 *     T_0 = 1,  T_{k+1} = T_k (1 - alpha_k),
 *     I = sum_k T_k alpha_k sigmoid(c_k) + T_N b,   A = 1 - T_N.
 * The background b (a colour, or one colour per pixel) is the Eq. (8) canvas term; A is the
 * alpha channel I_alpha of Supp. Alg. 1. The backward returns dL/dparams by the chain rule of
 * Eq. (7) and Supp. Eqs. (S4)-(S5).
 *
 * Conventions shared by every call:
 *   - params: device float32 [N, 8] row-major, columns x, y, log_s, theta, nu, c_r, c_g, c_b.
 *     x, y in pixels with pixel (px, py) at canvas point (px, py) (origin top-left, y down);
 *     s = exp(log_s) is the half-extent in pixels (Eq. 1 divides by s); theta in radians.
 *   - atlas_idx: device int32 [N], the bitmap of each primitive, in [0, B).
 *   - atlas: device [B, Hb, Wb] row-major, float32, bfloat16 or float16 (DBMP_F32, DBMP_BF16,
 *     DBMP_F16), values are template masks, normally in [0, 1]; Hb, Wb >= 2. Texels outside a
 *     bitmap read as 0. A float32 or bfloat16 atlas is sampled in float32. A float16 atlas
 *     selects the reduced-precision raster (the half-precision path of Sec. 3.1.2): each cell's
 *     texel pairs are fetched and bilinearly blended in packed fp16 (the blend's M, dM/dU' and
 *     dM/dV' carry fp16 rounding, about 3e-3 absolute for texels in [0, 1]); compositing,
 *     gradients and every accumulation stay in float32.
 *   - images are planar float32 [3, H, W]; alpha maps float32 [H, W].
 *   - every device pointer is owned by the caller and must stay valid (and unchanged) until the
 *     work queued on `stream` has finished; the library never frees caller memory.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream). Calls only enqueue work and
 *     return; none synchronises the host unless its comment says so.
 *   - return value: DBMP_OK or a negative dbmp_status. Argument errors are detected on the host
 *     and reported before anything is enqueued. Errors found on the device (an atlas index out
 *     of range, a non-finite parameter or texel, a full pair buffer) raise a flag in the context
 *     and are reported by dbmp_check(); the offending primitive is skipped, never read out of
 *     bounds. No exception ever crosses this interface.
 */
#ifndef DIFFBMP_H
#define DIFFBMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dbmp_ctx dbmp_ctx;
typedef void *dbmp_stream; /* hipStream_t */

typedef enum {
    DBMP_OK = 0,
    DBMP_EINVAL = -1,     /* bad argument (host check) or atlas index out of range (device) */
    DBMP_ENOMEM = -2,     /* device allocation failed */
    DBMP_EHIP = -3,       /* a HIP runtime call failed; dbmp_last_error() names it */
    DBMP_EOVERFLOW = -4,  /* more (tile, primitive) pairs than the pair buffer holds */
    DBMP_ESTATE = -5,     /* backward without a matching forward on this context */
    DBMP_ENONFINITE = -6  /* a parameter or atlas texel is NaN or infinite */
} dbmp_status;

typedef enum { DBMP_F32 = 0, DBMP_BF16 = 1, DBMP_F16 = 2 } dbmp_dtype;

#define DBMP_DEFAULT_TILE 16 /* the tile a call given tile = 0 uses */

/* Creates a context on HIP device `device`. The context owns the workspace (per-primitive
 * records, the per-tile primitive lists, the padded atlas and the per-pixel state the backward
 * needs) and grows it on demand. Every screen tile gets a list of `list_capacity` entries
 * (0 = a default of 256); a forward in which some tile is overlapped by more primitives raises
 * DBMP_EOVERFLOW (dbmp_check) and renders nothing. Synchronous. */
int dbmp_create(dbmp_ctx **out, int device, long long list_capacity);

/* Releases the context and its workspace. Synchronises the device first. */
int dbmp_destroy(dbmp_ctx *ctx);

/* Raises the per-tile list capacity to at least `list_capacity` entries (never lowers it; the
 * memory grows at the next forward) and restarts the dbmp_longest_list statistic. Synchronous.
 * Use after dbmp_check() returned DBMP_EOVERFLOW, with dbmp_longest_list() as the size. */
int dbmp_reserve(dbmp_ctx *ctx, long long list_capacity);

/*
 * Launch schedule of the raster kernels for the following forwards (and the backwards of those
 * forwards). Results do not depend on it: every tile is computed the same way; only which
 * workgroup computes it, and when, changes.
 *   DBMP_SCHED_GRID        one workgroup per screen tile, in image order (default).
 *   DBMP_SCHED_SORTED      one workgroup per tile, tiles dealt longest list first: by the list
 *                          lengths of the previous forward on this context (an extra binning
 *                          workgroup sorts them while the others bin; up to 4,096 tiles), or of
 *                          this forward (a counting sort after binning; more tiles). Any order is
 *                          valid: it only balances the compute units.
 *   DBMP_SCHED_PERSISTENT  workgroups_per_cu x (compute units) workgroups stay resident and take
 *                          tiles, longest list first: items_per_grab tiles at a time from a
 *                          device work queue until it is empty, or, with items_per_grab = 0,
 *                          every G-th tile of the order (G = the number of workgroups, no
 *                          atomics). One launch per stage however many images a batch holds.
 * workgroups_per_cu in [1, 32] and items_per_grab in [0, 1024] are used by
 * DBMP_SCHED_PERSISTENT only. Host-only, no synchronisation; the sorted schedules need a
 * workspace that grows at the next forward (not during graph capture).
 */
typedef enum { DBMP_SCHED_GRID = 0, DBMP_SCHED_SORTED = 1, DBMP_SCHED_PERSISTENT = 2 } dbmp_schedule;

int dbmp_set_schedule(dbmp_ctx *ctx, int schedule, int workgroups_per_cu, int items_per_grab);

/*
 * Where the raster kernels read texels (Sec. 3.1.2 stages primitive templates in on-chip shared
 * memory):
 *   DBMP_ATLAS_GLOBAL  the padded atlas in device memory, through the L1 and L2 caches (default);
 *   DBMP_ATLAS_LDS     every workgroup first copies the whole padded atlas,
 *                      B (Hb + 2)(Wb + 2) + 2 (Wb + 2) texels, into LDS and samples that copy;
 *                      taken by launches of the pipelined build (at most 16 waves per compute
 *                      unit: small canvases) when the copy takes at most
 *                      DBMP_ATLAS_LDS_MAX_BYTES; other launches read device memory.
 * Results are bit-identical either way (the gradient up to the order of its float atomics).
 * Host-only; applies to the forwards that follow (and their backwards).
 */
typedef enum { DBMP_ATLAS_GLOBAL = 0, DBMP_ATLAS_LDS = 1 } dbmp_atlas_placement;
#define DBMP_ATLAS_LDS_MAX_BYTES 32768
int dbmp_set_atlas_placement(dbmp_ctx *ctx, int placement);

/*
 * Measurement hook: the next raster kernel launch of `stage` on this context (0: the forward
 * compositing kernel of dbmp_render / dbmp_render_batched; 1: the backward kernel of
 * dbmp_render_backward / dbmp_render_backward_mse) is launched so that the device records
 * start_event when the kernel begins and stop_event when it ends (hipEvent_t handles created
 * by the caller with timing enabled; hipEventElapsedTime then gives the kernel's own duration).
 * One-shot; NULL, NULL disarms. Ignored for a launch made during graph capture.
 */
int dbmp_time_next_launch(dbmp_ctx *ctx, int stage, void *start_event, void *stop_event);

/*
 * Stores the bitmap templates in the context: each bitmap is copied with a one-texel zero border
 * (the zero padding of the bilinear sampler) and its bounding box of non-zero texels is found.
 * DBMP_EINVAL if the padded copy, B x (Hb + 2) x (Wb + 2) texels, would reach 4 GiB.
 * Renders given atlas == NULL use this copy, so a fit loop pays for it once. A render given an
 * atlas replaces it. Asynchronous on `stream`; the caller's atlas may be freed once the work on
 * `stream` has finished.
 */
int dbmp_set_atlas(dbmp_ctx *ctx, dbmp_stream stream, const void *atlas, int B, int Hb, int Wb,
                   int atlas_dtype);

/*
 * Forward render of one image (Eqs. 1-5 with background), Sec. 3.1.1.
 *   params, atlas_idx, N      primitives (see conventions); N >= 0 (N = 0 gives I = b, A = 0).
 *   atlas, B, Hb, Wb, dtype   bitmap templates, or atlas = NULL to use the context's atlas (set
 *                             by dbmp_set_atlas or a previous render; B, Hb, Wb, dtype ignored).
 *   H, W                      canvas size, >= 1.
 *   bg                        device float32: 3 values, or [3, H, W] when bg_per_pixel != 0.
 *   alpha_max                 in (0, 1] (Eq. 3).
 *   tile                      screen tile edge in pixels: 8, 16 or 32, or 0 for the library's
 *                             choice, DBMP_DEFAULT_TILE (the fastest on every measured workload,
 *                             128x128 to 2048x2048 and batches of uneven canvases; the Python
 *                             autotuner times the candidates for a given workload instead).
 *   image                     out, device float32 [3, H, W].
 *   alpha                     out, device float32 [H, W], A = 1 - T_N; may be NULL.
 * The context keeps what dbmp_render_backward needs (no per-layer state: the backward
 * recomputes transmittance per tile); params, atlas and bg must stay unchanged until then.
 */
int dbmp_render(dbmp_ctx *ctx, dbmp_stream stream, const float *params, const int32_t *atlas_idx,
                int N, const void *atlas, int B, int Hb, int Wb, int atlas_dtype, int H, int W,
                const float *bg, int bg_per_pixel, float alpha_max, int tile, float *image,
                float *alpha);

/*
 * Backward of the last dbmp_render / dbmp_render_batched on this context (Eq. 7, Supp. S4-S5).
 *   dL_dimage   device float32 [3, H, W] (batched: the concatenated layout of the forward).
 *   dL_dalpha   device float32 [H, W] or NULL (no loss on A).
 *   dL_dparams  out, device float32 [N, 8], overwritten (columns as in params; the scale
 *               column is dL/dlog_s).
 * Returns DBMP_ESTATE if no forward has run on this context.
 */
int dbmp_render_backward(dbmp_ctx *ctx, dbmp_stream stream, const float *dL_dimage,
                         const float *dL_dalpha, float *dL_dparams);

/*
 * Backward of the last forward for the loss L = mean((I - target)^2) over each image's 3HW values
 * (the `mse` loss of Supp. Table S1) plus any dL/dA: identical to dbmp_render_backward with
 * dL/dI = 2 (I - target) / (3 H W), but the gradient is formed inside the backward from the
 * forward's image instead of being read from a separate buffer.
 *   target      device float32, laid out like the forward's image.
 *   dL_dalpha   device float32 like the forward's alpha, or NULL.
 *   dL_dparams  out, device float32 [rows, 8], overwritten.
 *   accumulate  0: dL_dparams is overwritten; 1: the gradient is ADDED to dL_dparams (a fit
 *               loop whose optimiser zeroes the gradient after use saves a clearing pass).
 * The image passed to the forward must be unchanged. The squared errors are kept per tile for
 * dbmp_mse_loss. Returns DBMP_ESTATE if no forward has run on this context.
 */
int dbmp_render_backward_mse(dbmp_ctx *ctx, dbmp_stream stream, const float *target,
                             const float *dL_dalpha, float *dL_dparams, int accumulate);

/*
 * One fit step's render and MSE backward in one launch per stage (the forward of dbmp_render,
 * then in the same workgroups the backward of dbmp_render_backward_mse, reusing the image, the
 * per-pixel state and the staged primitive records while they are still on chip):
 *   arguments as dbmp_render (alpha is not produced), plus
 *   target       device float32 [3, H, W];
 *   image        out, the forward's image, as dbmp_render;
 *   dL_dparams   out, device float32 [N, 8]: dL/dparams of L = mean((I - target)^2), added to
 *                the buffer (accumulate != 0) or written (accumulate == 0).
 * Afterwards dbmp_mse_loss reports the loss and the context holds the state of a forward (a
 * later dbmp_render_backward* reuses it). Results equal those of the two separate calls (the
 * gradient up to the order of its float atomics).
 */
int dbmp_render_mse(dbmp_ctx *ctx, dbmp_stream stream, const float *params,
                    const int32_t *atlas_idx, int N, const void *atlas, int B, int Hb, int Wb,
                    int atlas_dtype, int H, int W, const float *bg, int bg_per_pixel,
                    float alpha_max, int tile, const float *target, float *image,
                    float *dL_dparams, int accumulate);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): dbmp_render_mse with no context. The workspace a
 * context would own lives in one static device array of DBMP_NOALLOC_SCRATCH_MB MiB per device,
 * held from the library's first use on that device until the process ends; the call allocates
 * and frees nothing. Results are those of dbmp_render_mse with the default schedule (the image
 * bit for bit, the gradient up to the order of its float atomics).
 *   arguments as dbmp_render_mse, on the current HIP device, with the atlas given every call;
 *   list_capacity  entries per tile list (>= 1; rounded up to a multiple of 32): the most
 *                  primitives that may overlap one screen tile;
 *   status         out, device int32 [4], cleared by the call, then {a tile list overflowed
 *                  (that tile is neither rendered nor differentiated), an atlas index out of
 *                  range, a non-finite parameter or texel, 0}: non-zero raises it;
 *   scratch_bytes  out, host, may be NULL: the scratch these sizes need (written also when the
 *                  call is refused).
 * DBMP_ENOMEM (nothing enqueued) if the sizes need more than the static array: about
 * 160 N + 4 n_tiles list_capacity + 8 H W + the padded atlas + 12 n_tiles bytes, so 2048 x 2048
 * with 65,536 primitives fits with list_capacity 96. DBMP_EINVAL for bad arguments (as
 * dbmp_render_mse), DBMP_EHIP if a launch failed. The first call on a device resolves the
 * array's address (hipGetSymbolAddress): make it outside graph capture. Every call on a device
 * uses that device's array, so calls that overlap in time on one device (other streams, other
 * host threads) race and must not be issued; consecutive calls on one stream are safe.
 */
#define DBMP_NOALLOC_SCRATCH_MB 64
int dbmp_render_mse_noalloc(dbmp_stream stream, const float *params, const int32_t *atlas_idx,
                            int N, const void *atlas, int B, int Hb, int Wb, int atlas_dtype,
                            int H, int W, const float *bg, int bg_per_pixel, float alpha_max,
                            int tile, int list_capacity, const float *target, float *image,
                            float *dL_dparams, int accumulate, int32_t *status,
                            size_t *scratch_bytes);

/* Sum over pixels and channels of (I - target)^2 of each image of the last
 * dbmp_render_backward_mse, written to out[0 .. n_images) (device float32). Asynchronous. */
int dbmp_mse_loss(dbmp_ctx *ctx, dbmp_stream stream, float *out);

/*
 * Batched forward: n_images independent images rendered by one launch per stage (binning, raster;
 * with DBMP_SCHED_PERSISTENT one resident grid drains all images' tiles).
 * Image i has desc[i] = {H, W, N, prim_offset, pixel_offset}: its primitives are rows
 * [prim_offset, prim_offset + N) of params / atlas_idx, its image occupies
 * image[3 * pixel_offset + c * H * W + y * W + x] and its alpha alpha[pixel_offset + y * W + x].
 * bg: 3 floats per image ([n_images, 3]). All images share the atlas, alpha_max and tile size.
 * `descs` is a HOST array; it is copied into the context before this call returns.
 */
typedef struct {
    int32_t H, W, N, reserved;
    int64_t prim_offset;
    int64_t pixel_offset;
} dbmp_image_desc;

int dbmp_render_batched(dbmp_ctx *ctx, dbmp_stream stream, int n_images,
                        const dbmp_image_desc *descs, const float *params,
                        const int32_t *atlas_idx, const void *atlas, int B, int Hb, int Wb,
                        int atlas_dtype, const float *bg, float alpha_max, int tile,
                        float *image, float *alpha);

/* dbmp_render_mse over a batch of images (dbmp_render_batched's layout; each image's loss is the
 * mean over its own 3HW values). */
int dbmp_render_batched_mse(dbmp_ctx *ctx, dbmp_stream stream, int n_images,
                            const dbmp_image_desc *descs, const float *params,
                            const int32_t *atlas_idx, const void *atlas, int B, int Hb, int Wb,
                            int atlas_dtype, const float *bg, float alpha_max, int tile,
                            const float *target, float *image, float *dL_dparams,
                            int accumulate);

/*
 * One Adam iteration of a fit (the MSE loss and Adam optimiser of Supp. Table S1) in two
 * launches instead of three: the binning first applies to `params` the Adam update of the
 * gradient the previous call left in `grad` (if `state` marks one pending), clearing it, and
 * bins the updated parameters; the fused forward + MSE backward of dbmp_render_mse then adds
 * the new gradient into `grad` and marks it pending. The stored atlas is used (dbmp_set_atlas).
 *   params       in/out, device float32 [N, 8].
 *   grad, m, v   device float32 [N, 8]: the pending gradient and Adam's moments; grad must hold
 *                zeros before the first call.
 *   state        device int32 [4]: {updates applied t, unused, gradient pending, unused}, zeros
 *                before the first call (the fused launch counts the update the binning applied
 *                and marks its own gradient pending).
 *   lr, beta1, beta2, eps  Adam's hyper-parameters (as dbmp_adam_step).
 *   other arguments as dbmp_render_mse; image receives the forward's image.
 * Update j computes exactly what dbmp_adam_step computes with the same t and zero_grad = 1. After
 * the last call, dbmp_adam_step(..., state, zero_grad = 1) applies the pending gradient (then
 * clear state[2]). dbmp_mse_loss reports the loss of the image rendered by the last call.
 */
int dbmp_fit_step(dbmp_ctx *ctx, dbmp_stream stream, float *params, const int32_t *atlas_idx,
                  int N, int H, int W, const float *bg, int bg_per_pixel, float alpha_max,
                  int tile, const float *target, float *image, float *grad, float *m, float *v,
                  int32_t *state, float lr, float beta1, float beta2, float eps);

/* dbmp_fit_step over a batch of images (dbmp_render_batched's layout; each image's loss is the
 * mean over its own 3HW values; Adam updates every row below the largest prim_offset + N). */
int dbmp_fit_step_batched(dbmp_ctx *ctx, dbmp_stream stream, int n_images,
                          const dbmp_image_desc *descs, float *params, const int32_t *atlas_idx,
                          const float *bg, float alpha_max, int tile, const float *target,
                          float *image, float *grad, float *m, float *v, int32_t *state, float lr,
                          float beta1, float beta2, float eps);

/* Synchronises `stream` and reports the device-side errors raised by any forward since the
 * previous dbmp_check: DBMP_EOVERFLOW (a tile list did not fit; that forward's image is not
 * valid), DBMP_EINVAL (atlas index out of range), DBMP_ENONFINITE, or DBMP_OK. The reported
 * errors are cleared. */
int dbmp_check(dbmp_ctx *ctx, dbmp_stream stream);

/* Longest tile list (number of primitives overlapping one screen tile) of all forwards since
 * the last dbmp_reserve (or dbmp_create): the capacity to pass to dbmp_reserve after
 * DBMP_EOVERFLOW. Synchronises `stream`. */
long long dbmp_longest_list(dbmp_ctx *ctx, dbmp_stream stream);

/* Number of (pixel, primitive) pairs evaluated by all forwards on this context since it was
 * created or last reset: pairs where the primitive's bilinear footprint at the pixel reads at
 * least one non-zero texel (elsewhere M and its derivatives are exactly zero, Supp. Eqs. S1-S3).
 * Synchronises `stream`; reset != 0 zeroes the count afterwards (synchronously). -1 on error. */
long long dbmp_support_pairs(dbmp_ctx *ctx, dbmp_stream stream, int reset);

/* Number of times the context's workspace has been reallocated so far (-1 for a NULL context).
 * The workspace grows (synchronously, outside graph capture) when a call needs more room than any
 * earlier one: a larger canvas, more primitives or tiles, a larger list capacity or atlas. A growth
 * releases the old memory, so a HIP graph captured on this context before it refers to freed
 * addresses and must be captured again; compare the epoch at capture and before a replay. */
long long dbmp_workspace_epoch(const dbmp_ctx *ctx);

/* Device bytes the context's workspace holds now (records, tile lists and counters, the per-pixel
 * (K, T_K), the padded atlas, descriptors and flags); -1 for a NULL context. Memory the caller
 * passes in (parameters, images, gradients) is not included. */
long long dbmp_workspace_bytes(const dbmp_ctx *ctx);

/* Message of the last error on this context ("" if none). Valid until the next call. */
const char *dbmp_last_error(const dbmp_ctx *ctx);

/*
 * Mean-squared-error gradient over n values (the `mse` loss of the paper's configuration, Supp.
 * Table S1): grad[i] = 2 (image[i] - target[i]) / n. If loss != NULL it points to THREE device
 * float32 (zero before the first call; [1] and [2] are scratch the call leaves at zero) and
 * loss[0] receives sum_i (image[i] - target[i])^2.
 */
int dbmp_mse_grad(dbmp_stream stream, const float *image, const float *target, long long n,
                  float *grad, float *loss);

/*
 * One Adam step (Kingma & Ba, Algorithm 1; the optimiser of Supp. Table S1 with a flat rate) on
 * n float32 values in place: m, v are the moment buffers (zero before the first step). `step`
 * points to TWO device int32: step[0] counts the steps already taken and step[1] is scratch for
 * the kernel; both must be zero before the first step. The call uses t = step[0] + 1 for the
 * bias correction and advances step[0] on the device, so it can be replayed from a graph.
 * zero_grad != 0 sets grad to zero after reading it (for an accumulating backward).
 */
int dbmp_adam_step(dbmp_stream stream, float *params, float *grad, float *m, float *v,
                   long long n, float lr, float beta1, float beta2, float eps, int32_t *step,
                   int zero_grad);

#ifdef __cplusplus
}
#endif

#endif /* DIFFBMP_H */
