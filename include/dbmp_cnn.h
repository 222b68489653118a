/*
 * C ABI of the learned initialiser's kernels (libdiffbmp.so): the layers of a small CNN that
 * predicts primitive parameters from a target image, in bfloat16 with float32 accumulation on
 * the matrix cores (the "learned parts" of the method: an initialiser trained on pairs of
 * (target, parameters fitted by the plain optimiser), with the plain random initialisation kept
 * as fallback).
 *
 * Conventions.
 *   - bf16 tensors are passed as uint16_t bit patterns. Activations are NHWC: [B][H][W][C].
 *   - Convolutions are 3x3, stride 2, zero padding 1: an H x W input gives H/2 x W/2 (H, W
 *     even). Weights are [Cout][3][3][Cin] (float32 master copies of the same layout are cast
 *     by dbmp_cnn_cast_weights); the gradient with respect to the input reads a transposed copy
 *     [Cin][3][3][Cout].
 *   - Dense layers: x [B][K], weights [N][K], transposed copy [K][N].
 *   - Channel counts that are read 8 at a time must be multiples of 8 (stated per call).
 *   - Gradients with respect to weights and biases are ADDED into float32 buffers (zero them,
 *     or let the optimiser zero them, between steps).
 *   - All calls are asynchronous on `stream` (a hipStream_t); every pointer is device memory
 *     owned by the caller. Returns DBMP_CNN_OK, DBMP_CNN_EINVAL (bad argument, nothing
 *     launched) or DBMP_CNN_EHIP (a launch failed).
 */
#ifndef DBMP_CNN_H
#define DBMP_CNN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { DBMP_CNN_OK = 0, DBMP_CNN_EINVAL = -1, DBMP_CNN_EHIP = -3 };

/* y[b][oy][ox][oc] = act(bias[oc] + sum_{ky,kx,ic} w[oc][ky][kx][ic] x[b][2oy+ky-1][2ox+kx-1][ic])
 * with act = ReLU if relu != 0. Cin % 8 == 0. y (bf16) and/or y32 (float32) may be NULL (not
 * both); bias may be NULL. */
int dbmp_cnn_conv_forward(void *stream, const uint16_t *x, int B, int H, int W, int Cin,
                          const uint16_t *w, const float *bias, int Cout, int relu, uint16_t *y,
                          float *y32);

/* dx[b][y][x][ic] = [mask > 0] * sum over (ky, kx, oc) with y = 2oy+ky-1, x = 2ox+kx-1 of
 * wt[ic][ky][kx][oc] dz[b][oy][ox][oc]; mask (the layer's input activation, whose producing
 * ReLU the gradient passes through) may be NULL. H, W are the INPUT size. Cin, Cout % 8 == 0. */
int dbmp_cnn_conv_backward_data(void *stream, const uint16_t *dz, int B, int H, int W, int Cin,
                                const uint16_t *wt, int Cout, const uint16_t *mask,
                                uint16_t *dx);

/* dw[oc][ky][kx][ic] += sum_{b,oy,ox} dz[b][oy][ox][oc] x[b][2oy+ky-1][2ox+kx-1][ic] and, if db
 * is not NULL, db[oc] += sum_{b,oy,ox} dz[b][oy][ox][oc]. H, W are the input size. */
int dbmp_cnn_conv_backward_weight(void *stream, const uint16_t *x, const uint16_t *dz, int B,
                                  int H, int W, int Cin, int Cout, float *dw, float *db);

/* y[b][n] = act(bias[n] + sum_k w[n][k] x[b][k]); K % 8 == 0. */
int dbmp_cnn_linear_forward(void *stream, const uint16_t *x, int B, int K, const uint16_t *w,
                            const float *bias, int N, int relu, uint16_t *y, float *y32);

/* dx[b][k] = [mask > 0] * sum_n wt[k][n] dz[b][n]; N % 8 == 0; mask may be NULL. */
int dbmp_cnn_linear_backward_data(void *stream, const uint16_t *dz, int B, int N,
                                  const uint16_t *wt, int K, const uint16_t *mask, uint16_t *dx);

/* dw[n][k] += sum_b dz[b][n] x[b][k]; db[n] += sum_b dz[b][n] (db may be NULL). */
int dbmp_cnn_linear_backward_weight(void *stream, const uint16_t *x, const uint16_t *dz, int B,
                                    int K, int N, float *dw, float *db);

/* bf16 copies of float32 weights w [R][T][C]: wb in the same layout and wt in [C][T][R]
 * (either may be NULL). Convolutions: R = Cout, T = 9, C = Cin; dense: R = N, T = 1, C = K. */
int dbmp_cnn_cast_weights(void *stream, const float *w, int R, int T, int C, uint16_t *wb,
                          uint16_t *wt);

/* float32 planar RGB images [B][3][H][W] -> bf16 NHWC [B][H][W][8], channels 3..7 zero. */
int dbmp_cnn_pack_input(void *stream, const float *img, int B, int H, int W, uint16_t *x);

/* Regression loss on rows of 8 parameters, n values (n % 8 == 0): column q contributes
 * weights8[q] (pred - target)^2, except the angle column 3, which contributes
 * weights8[3] (1 - cos(pred - target)). Writes, as bf16,
 *     dpred[i] = scale * dL/dpred[i] + extra[i] * extra_scale8[i % 8]
 * (target may be NULL: no regression term; extra may be NULL: no added gradient; it carries a
 * gradient that reaches the predictions from elsewhere, e.g. an image loss through the
 * renderer, and extra_scale8 is a HOST array of 8 factors). Adds scale * L to *loss (float32;
 * may be NULL). */
int dbmp_cnn_param_loss(void *stream, const float *pred, const float *target,
                        const float *weights8, long long n, float scale, const float *extra,
                        const float *extra_scale8, uint16_t *dpred, float *loss);

/* Per-column affine coding of n_rows parameter rows [n_rows][8], row r being slot r % slots of
 * a grid x grid template with cells of `cell` pixels. Slots are numbered one block of
 * block x block cells at a time: slot k is cell (k % block^2) (row-major) of block
 * k / block^2, the blocks taken row-major over the grid (block = 1: the cells row-major;
 * block must divide grid). With centre(r, q) the slot's cell centre for q = 0 (x) and q = 1 (y)
 * and 0 otherwise, and clip() limiting every column but the angle (3) to [-clip, clip],
 *     decode != 0:  out = clip(in) * scale8[q] + bias8[q] + centre(r, q)
 *     decode == 0:  out = clip((in - bias8[q] - centre(r, q)) / scale8[q]).
 * scale8 and bias8 are HOST arrays (scale8[q] != 0). in and out may not overlap. */
int dbmp_cnn_code_params(void *stream, const float *in, long long n_rows, int slots, int grid,
                         int block, float cell, const float *scale8, const float *bias8,
                         float clip, int decode, float *out);

#ifdef __cplusplus
}
#endif

#endif /* DBMP_CNN_H */
