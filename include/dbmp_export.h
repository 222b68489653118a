/*
 * dbmp_export.h -- C ABI of the layer export (DiffBMP, arXiv 2602.22625, Sec. 3.1.3 and Supp.
 * "PSD export"), for gfx950: every primitive rendered alone into its own layer, at an export
 * scale rho (e.g. 2 or 4: the optimisation runs at a low resolution, the layers are written at a
 * higher one), with primitive-level parallelism and no atomics. A layer is the primitive's
 * constant colour sigmoid(c) and its alpha alpha_max sigmoid(nu) M(x, y) (Eqs. 1-3) over a box
 * of export pixels; composited front to back with the over operator (Eqs. 4-5) the layers give
 * the render at that scale.
 *
 * Export pixel (X, Y) covers the canvas point ((X + 0.5) / rho - 0.5, (Y + 0.5) / rho - 0.5):
 * the export grid spans the same canvas as the H x W one, with rho x rho export pixels per pixel.
 * The export canvas is round(rho H) x round(rho W).
 *
 * Conventions as in diffbmp.h (device pointers owned by the caller, parameter rows [N, 8],
 * atlas [B, Hb, Wb] float32, bfloat16 or float16). Calls only enqueue work on `stream`.
 */
#ifndef DBMP_EXPORT_H
#define DBMP_EXPORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *dbmp_export_stream; /* hipStream_t */

/*
 * Stage 1: per primitive, the box of export pixels that can hold a non-zero alpha (the image of
 * the bitmap's bilinear support, -1 < U < Wb and -1 < V < Hb, clipped to the export canvas):
 *   boxes    out, device int32 [N, 4] = x0, y0, w, h (w = h = 0: the layer is empty, also for a
 *            non-finite parameter row);
 *   offsets  out, device int64 [N + 1]: offsets[i] = sum of w h over the primitives before i,
 *            offsets[N] = the total (the alpha buffer's length for stage 2);
 *   max_wh   out, device int32 [2]: the largest w and the largest h.
 */
int dbmp_export_boxes(dbmp_export_stream stream, const float *params, int N, int Hb, int Wb,
                      int H, int W, double rho, int32_t *boxes, long long *offsets,
                      int32_t *max_wh);

/*
 * Stage 2: every layer's alpha, row-major over its box, at alpha_out[offsets[i] ..
 * offsets[i] + w h) (device float32, offsets[N] values), and its colour sigmoid(c) at
 * colour_out[3 i .. 3 i + 3) (device float32 [N, 3]). boxes, offsets: stage 1's output;
 * max_w, max_h: its max_wh (read back by the caller, which also sizes alpha_out).
 */
int dbmp_export_layers(dbmp_export_stream stream, const float *params, const int32_t *atlas_idx,
                       int N, const void *atlas, int B, int Hb, int Wb, int atlas_dtype, int H,
                       int W, double rho, float alpha_max, const int32_t *boxes,
                       const long long *offsets, int max_w, int max_h, float *alpha_out,
                       float *colour_out);

#ifdef __cplusplus
}
#endif

#endif /* DBMP_EXPORT_H */
