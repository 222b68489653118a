// Layer export (Sec. 3.1.3; Supp. "PSD export"), declared in include/dbmp_export.h.
//
// Stage 1: one lane per primitive finds the box of export pixels its bilinear support can reach
// (float64, as the binning), then one workgroup turns the box areas into offsets (an exclusive
// int64 scan). Stage 2: one workgroup per primitive walks its box's export pixels; each lane
// evaluates a pixel's alpha (the forward's arithmetic: float64 coordinates, float32 bilinear
// sample) and writes it into the primitive's own packed box. Every output value has exactly one
// writer, so no atomics.
#include "dbmp_export.h"
#include "dbmp_internal.h"
#include "diffbmp.h"

#include <limits.h>
#include <math.h>

namespace dbmp {
namespace {

// Canvas point of export pixel X: (X + 0.5) / rho - 0.5; export coordinate of canvas point x:
// rho (x + 0.5) - 0.5.
__global__ void __launch_bounds__(256)
k_export_boxes(const float *__restrict__ params, int N, int Hb, int Wb, int HH, int WW,
               double rho, int *__restrict__ boxes, long long *__restrict__ area,
               int *__restrict__ max_wh)
{
    const int i0 = blockIdx.x * 256 + threadIdx.x;
    const int i = i0 < N ? i0 : N - 1;  // lanes past N repeat the last row (no store below)
    const float *p = params + (size_t)i * 8;
    bool fin = true;
    for (int q = 0; q < 8; ++q) fin = fin && isfinite(p[q]);
    int x0 = 0, y0 = 0, w = 0, h = 0;
    const double s = exp((double)p[2]);
    if (fin && s > 0.0 && isfinite(s)) {
        double st, ct;
        sincos((double)p[3], &st, &ct);
        const double cu = 0.5 * (Wb - 1), cv = 0.5 * (Hb - 1);
        double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
        for (int c = 0; c < 4; ++c) {  // corners of -1 <= U <= Wb, -1 <= V <= Hb
            const double U = (c & 1) ? (double)Wb : -1.0, V = (c & 2) ? (double)Hb : -1.0;
            const double u = U / cu - 1.0, v = V / cv - 1.0;
            const double X = rho * ((double)p[0] + s * (ct * u - st * v) + 0.5) - 0.5;
            const double Y = rho * ((double)p[1] + s * (st * u + ct * v) + 0.5) - 0.5;
            xmin = fmin(xmin, X); xmax = fmax(xmax, X);
            ymin = fmin(ymin, Y); ymax = fmax(ymax, Y);
        }
        const double mg = 1e-3;  // conservative against rounding
        const double fx0 = fmax(ceil(xmin - mg), 0.0), fx1 = fmin(floor(xmax + mg), WW - 1.0);
        const double fy0 = fmax(ceil(ymin - mg), 0.0), fy1 = fmin(floor(ymax + mg), HH - 1.0);
        if (fx0 <= fx1 && fy0 <= fy1) {
            x0 = (int)fx0; y0 = (int)fy0;
            w = (int)(fx1 - fx0) + 1; h = (int)(fy1 - fy0) + 1;
        }
    }
    if (i0 < N) {
        boxes[4 * i + 0] = x0; boxes[4 * i + 1] = y0; boxes[4 * i + 2] = w; boxes[4 * i + 3] = h;
        area[i] = (long long)w * h;
    }
    // the largest box: a wave maximum, then one atomic per wave (one per lane on the same two
    // addresses would serialise)
    for (int o = 32; o > 0; o >>= 1) {
        w = max(w, __shfl_xor(w, o));
        h = max(h, __shfl_xor(h, o));
    }
    if ((threadIdx.x & 63) == 0 && w) { atomicMax(max_wh, w); atomicMax(max_wh + 1, h); }
}

__global__ void k_export_init(int *max_wh)
{
    max_wh[0] = 0;
    max_wh[1] = 0;
}

// Exclusive scan of the N areas into offsets[0 .. N] by one workgroup of 1024 lanes.
__global__ void __launch_bounds__(1024) k_export_offsets(long long *__restrict__ off, int N)
{
    __shared__ long long wsum[16];
    __shared__ long long carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int b0 = 0; b0 < N; b0 += 1024) {
        const int i = b0 + threadIdx.x;
        const long long x = i < N ? off[i] : 0;
        long long incl = x;
        for (int o = 1; o < 64; o <<= 1) {
            const long long y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        long long pre = carry;
        for (int q = 0; q < wave; ++q) pre += wsum[q];
        __syncthreads();
        if (i < N) off[i] = pre + incl - x;
        if (threadIdx.x == 1023) carry = pre + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) off[N] = carry;
}

template <typename TexT>
__device__ __forceinline__ float tex_at(const TexT *__restrict__ bm, int Hb, int Wb, int r, int c)
{
    return (r >= 0 && r < Hb && c >= 0 && c < Wb) ? texel<TexT>(bm[(size_t)r * Wb + c]) : 0.f;
}

// One workgroup per primitive: the primitive's constants once, then its box's pixels in
// row-major order, 256 at a time (coalesced stores into its packed box). A grid of (primitive,
// tile row, tile column) sized by the largest box launched mostly empty workgroups and
// evaluated the exponentials per pixel: 5.1 ms at 2048^2 with 65,536 primitives against
// 0.59 ms. (One wave per primitive took 1.17 ms: the largest boxes then run on 64 lanes.)
template <typename TexT>
__global__ void __launch_bounds__(256)
k_export_layers(const float *__restrict__ params, const int *__restrict__ idx, int B,
                const TexT *__restrict__ atlas, int Hb, int Wb, double rho, float alpha_max,
                const int *__restrict__ boxes, const long long *__restrict__ offsets,
                float *__restrict__ alpha_out, float *__restrict__ colour_out)
{
    const int i = blockIdx.x;
    const int bw = boxes[4 * i + 2], bh = boxes[4 * i + 3];
    const float *p = params + (size_t)i * 8;
    if (threadIdx.x < 3)
        colour_out[3 * i + threadIdx.x] = (float)(1.0 / (1.0 + exp(-(double)p[5 + threadIdx.x])));
    const int n = bw * bh;
    if (n == 0) return;
    float *out = alpha_out + offsets[i];
    const int k = idx[i];
    if (!(k >= 0 && k < B)) {
        for (int j = threadIdx.x; j < n; j += 256) out[j] = 0.f;
        return;
    }
    // the forward's map (float64), folded as the binning folds it: U = aU x + bU y + eU with
    // U = cu (u + 1), u = (cos dx + sin dy) / s (unpadded bitmap coordinates here)
    const double s = exp((double)p[2]);
    double st, ct;
    sincos((double)p[3], &st, &ct);
    const double cu = 0.5 * (Wb - 1), cv = 0.5 * (Hb - 1), inv_s = 1.0 / s;
    const double aU = cu * ct * inv_s, bU = cu * st * inv_s;
    const double aV = -cv * st * inv_s, bV = cv * ct * inv_s;
    const double px = p[0], py = p[1];
    const double eU = cu - aU * px - bU * py, eV = cv - aV * px - bV * py;
    const float ka = (float)((double)alpha_max / (1.0 + exp(-(double)p[4])));
    const double x0 = boxes[4 * i] + 0.5, y0 = boxes[4 * i + 1] + 0.5, ir = 1.0 / rho;
    const TexT *bm = atlas + (size_t)k * Hb * Wb;
    for (int j = threadIdx.x; j < n; j += 256) {
        const int by = j / bw, bx = j - by * bw;
        float a = 0.f;
        // canvas point of export pixel (X, Y): (X + 0.5) / rho - 0.5
        const double x = fma(x0 + bx, ir, -0.5), y = fma(y0 + by, ir, -0.5);
        const double U = fma(aU, x, fma(bU, y, eU));
        const double V = fma(aV, x, fma(bV, y, eV));
        const double u0 = floor(U), v0 = floor(V);
        if (u0 >= -1.0 && u0 <= Wb - 1.0 && v0 >= -1.0 && v0 <= Hb - 1.0) {
            const int iu = (int)u0, iv = (int)v0;
            const float wu = (float)(U - u0), wv = (float)(V - v0);
            const float p00 = tex_at(bm, Hb, Wb, iv, iu), p01 = tex_at(bm, Hb, Wb, iv, iu + 1);
            const float p10 = tex_at(bm, Hb, Wb, iv + 1, iu), p11 = tex_at(bm, Hb, Wb, iv + 1, iu + 1);
            const float top = fmaf(wu, p01 - p00, p00), bot = fmaf(wu, p11 - p10, p10);
            const float M = fmaf(wv, bot - top, top);
            a = ka * M;
        }
        out[j] = a;
    }
}

int launched() { return hipGetLastError() == hipSuccess ? DBMP_OK : DBMP_EHIP; }

bool export_canvas(int H, int W, double rho, int *HH, int *WW)
{
    if (H < 1 || W < 1 || !(rho > 0.0 && rho <= 64.0)) return false;
    const double hh = nearbyint(H * rho), ww = nearbyint(W * rho);
    if (hh < 1 || ww < 1 || hh * ww >= (double)INT_MAX) return false;
    *HH = (int)hh;
    *WW = (int)ww;
    return true;
}

}  // namespace
}  // namespace dbmp

using namespace dbmp;

extern "C" {

int dbmp_export_boxes(dbmp_export_stream stream, const float *params, int N, int Hb, int Wb,
                      int H, int W, double rho, int32_t *boxes, long long *offsets,
                      int32_t *max_wh)
{
    int HH = 0, WW = 0;
    if (N < 0 || Hb < 2 || Wb < 2 || !export_canvas(H, W, rho, &HH, &WW)) return DBMP_EINVAL;
    if (!offsets || !max_wh || (N > 0 && (!params || !boxes))) return DBMP_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    k_export_init<<<1, 1, 0, st>>>(max_wh);
    if (N > 0)
        k_export_boxes<<<(N + 255) / 256, 256, 0, st>>>(params, N, Hb, Wb, HH, WW, rho, boxes,
                                                       offsets, max_wh);
    k_export_offsets<<<1, 1024, 0, st>>>(offsets, N);
    return launched();
}

int dbmp_export_layers(dbmp_export_stream stream, const float *params, const int32_t *atlas_idx,
                       int N, const void *atlas, int B, int Hb, int Wb, int atlas_dtype, int H,
                       int W, double rho, float alpha_max, const int32_t *boxes,
                       const long long *offsets, int max_w, int max_h, float *alpha_out,
                       float *colour_out)
{
    int HH = 0, WW = 0;
    if (N < 0 || B < 1 || Hb < 2 || Wb < 2 || !export_canvas(H, W, rho, &HH, &WW))
        return DBMP_EINVAL;
    if (atlas_dtype != DBMP_F32 && atlas_dtype != DBMP_BF16 && atlas_dtype != DBMP_F16)
        return DBMP_EINVAL;
    if (!(alpha_max > 0.f && alpha_max <= 1.f)) return DBMP_EINVAL;
    if (max_w < 0 || max_h < 0 || max_w > WW || max_h > HH) return DBMP_EINVAL;
    if (N == 0) return DBMP_OK;
    if (!params || !atlas_idx || !atlas || !boxes || !offsets || !colour_out) return DBMP_EINVAL;
    if (max_w > 0 && !alpha_out) return DBMP_EINVAL;
    const dim3 grid(N);
    hipStream_t st = (hipStream_t)stream;
    if (atlas_dtype == DBMP_F32)
        k_export_layers<float><<<grid, 256, 0, st>>>(
            params, atlas_idx, B, (const float *)atlas, Hb, Wb, rho, alpha_max, boxes, offsets,
            alpha_out, colour_out);
    else if (atlas_dtype == DBMP_F16)
        k_export_layers<_Float16><<<grid, 256, 0, st>>>(
            params, atlas_idx, B, (const _Float16 *)atlas, Hb, Wb, rho, alpha_max, boxes, offsets,
            alpha_out, colour_out);
    else
        k_export_layers<uint16_t><<<grid, 256, 0, st>>>(
            params, atlas_idx, B, (const uint16_t *)atlas, Hb, Wb, rho, alpha_max, boxes, offsets,
            alpha_out, colour_out);
    return launched();
}

}  // extern "C"
