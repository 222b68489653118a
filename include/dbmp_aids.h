/*
 * dbmp_aids.h -- C ABI of the optimisation aids around the rasteriser (DiffBMP, arXiv
 * 2602.22625, Sec. 3.2 and Eqs. 8-9; Supp. Table S1 and Sec. S1.4.2), for gfx950.
 *
 * Conventions as in diffbmp.h: device pointers owned by the caller, planar float32 images
 * [3, H, W], alpha maps [H, W], parameter rows [N, 8] = x, y, log_s, theta, nu, c_r, c_g, c_b;
 * every call only enqueues work on `stream` (a hipStream_t) and returns DBMP_OK or a negative
 * dbmp_status (DBMP_EINVAL for bad arguments, checked on the host before anything is enqueued;
 * DBMP_EHIP if a launch failed). Random numbers a step draws are inputs (device arrays the
 * caller fills), except the noise canvas, which runs its own counter-based generator.
 */
#ifndef DBMP_AIDS_H
#define DBMP_AIDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *dbmp_aids_stream; /* hipStream_t */

/*
 * Soft rasterisation (Sec. 3.2.1; blur_sigma = 1 in Supp. Table S1): every bitmap of the atlas
 * convolved with a Gaussian of standard deviation `sigma` texels, taps d = -r..r with
 * r = floor(truncate * sigma + 0.5) (truncate = 3 is the usual cut), normalised to sum 1;
 * texels outside the bitmap read 0 and the bitmap keeps its size. Separable, float32.
 *   atlas  device [B, Hb, Wb], DBMP_F32, DBMP_BF16 or DBMP_F16 (diffbmp.h); out: same layout
 *          and dtype, must not overlap atlas (bf16 and f16 results rounded to nearest even).
 * sigma in (0, 8], r <= 16, Wb <= 1024.
 */
int dbmp_blur_atlas(dbmp_aids_stream stream, const void *atlas, int B, int Hb, int Wb,
                    int atlas_dtype, float sigma, float truncate, void *out);

/* Bytes of device workspace dbmp_sa_init needs for an H x W target. */
long long dbmp_sa_init_workspace_bytes(int H, int W);

/*
 * Structure-aware initialisation (Sec. 3.2.2): N primitives placed where the target is complex.
 *   1. LV(x, y): per channel, the variance of the target over the win x win window centred on
 *      the pixel (clipped at the border), averaged over the channels (float64).
 *   2. NLV = (LV - min LV) / (max LV - min LV) (zeros for a flat target), written to nlv_out
 *      (device float32 [H, W]).
 *   3. Every lattice point (pixel) gets the integer weight floor((base + (1 - base) NLV) 2^24)
 *      (base = 0.1 in the paper), computed in float64 from the float32 NLV; primitive i takes
 *      the first pixel p whose cumulative weight exceeds floor(u_pos[i] * total) (exact int64
 *      sums, so the draw does not depend on the order of the sums).
 *   4. Its row of params_out (device float32 [N, 8]): x = p mod W, y = p div W,
 *      log s = log(s_max - (s_max - s_min) NLV(p)), theta = 2 pi u_theta[i], nu = nu_init,
 *      colour logits of clip(target(p) + sigma_c z_col[i], 1e-3, 1 - 1e-3).
 *   target       device float32 [3, H, W]; win odd in [1, 15].
 *   u_pos, u_theta  device float32 [N], uniforms in [0, 1); z_col device float32 [N, 3], N(0, 1).
 *   workspace    device, at least dbmp_sa_init_workspace_bytes(H, W) bytes, 16-byte aligned.
 */
int dbmp_sa_init(dbmp_aids_stream stream, const float *target, int H, int W, int win,
                 double base, const float *u_pos, const float *u_theta, const float *z_col, int N,
                 double s_min, double s_max, double nu_init, double sigma_c, void *workspace,
                 long long workspace_bytes, float *nlv_out, float *params_out);

/*
 * Uniform-noise canvas of Eq. (8), one draw per iteration: bg_out (device float32 [3, H, W]) at
 * pixel p = y W + x takes the Philox4x64-10 block (Salmon et al., SC 2011) of counter
 * (p, iteration, 0, 0) and key (seed, 0); its words 0, 1, 2 give red, green and blue as
 * (word >> 40) * 2^-24, uniform in [0, 1). Pass bg_out as the per-pixel background of a render.
 */
int dbmp_noise_canvas(dbmp_aids_stream stream, unsigned long long seed,
                      unsigned long long iteration, int H, int W, float *bg_out);

/*
 * Spatial-constraint objective of Eq. (9), as means:
 *   L = mean_{3HW} [A_t > 0] (I - I_t)^2 + lambda mean_{HW} (A - A_t)^2,
 * its gradients dL_dimage [3, H, W] and dL_dalpha [H, W] (overwritten; pass them to
 * dbmp_render_backward), and L added to loss[0] (device float32, may be NULL).
 *   image, target [3, H, W]; alpha, target_alpha [H, W]: device float32.
 */
int dbmp_constraint_loss(dbmp_aids_stream stream, const float *image, const float *alpha,
                         const float *target, const float *target_alpha, int H, int W,
                         float lambda, float *dL_dimage, float *dL_dalpha, float *loss);

/*
 * Re-initialisation of transparent primitives (Supp. Sec. S1.4.2): every row whose opacity
 * sigmoid(nu) is below `threshold` (decided as nu < logit(threshold) in float64) is replaced
 * by the same row of `proposal` (a fresh dbmp_sa_init draw), and its Adam moments m, v are
 * zeroed (m, v may be NULL). count (device int32, may be NULL) is increased by the number of
 * rows replaced. params, m, v, proposal: device float32 [N, 8]; threshold in (0, 1).
 */
int dbmp_reinit_transparent(dbmp_aids_stream stream, float *params, float *m, float *v,
                            const float *proposal, int N, double threshold, int32_t *count);

#ifdef __cplusplus
}
#endif

#endif /* DBMP_AIDS_H */
