// Optimisation aids around the rasteriser (Sec. 3.2, Eqs. 8-9; Supp. Table S1, Sec. S1.4.2):
// Gaussian blur of the bitmaps, structure-aware initialisation, the noise canvas, the
// spatial-constraint loss and the re-initialisation of transparent primitives. Declared in
// include/dbmp_aids.h. All of it is elementwise, stencil or scan work: bound by memory, laid out
// for coalesced rows, with LDS staging where a value is read by many neighbours.
#include "dbmp_aids.h"
#include "dbmp_internal.h"
#include "diffbmp.h"

#include <limits.h>
#include <algorithm>
#include <math.h>

namespace dbmp {
namespace {

// ------------------------------------------------------------------------------------------
// Gaussian blur (Sec. 3.2.1): a band of output rows per workgroup. The band's input rows plus
// r rows above and below are staged in LDS (as float32), blurred along x into a second LDS
// buffer, then along y into the output: each input texel is read from HBM once per band.
// ------------------------------------------------------------------------------------------
constexpr int BLUR_RMAX = 16;
constexpr int BLUR_LDS_BYTES = 48 * 1024;

struct BlurTaps {
    float w[2 * BLUR_RMAX + 1];
    int r;
};

template <typename TexT> __device__ __forceinline__ TexT from_f32(float v);
template <> __device__ __forceinline__ float from_f32<float>(float v) { return v; }
template <> __device__ __forceinline__ uint16_t from_f32<uint16_t>(float v)
{
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)0x7fc0;  // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                // round to nearest even
    return (uint16_t)(u >> 16);
}
template <> __device__ __forceinline__ _Float16 from_f32<_Float16>(float v)
{
    return (_Float16)v;  // round to nearest even
}

template <typename TexT>
__global__ void __launch_bounds__(256)
k_blur(const TexT *__restrict__ in, TexT *__restrict__ out, int Hb, int Wb, int band, BlurTaps t)
{
    extern __shared__ float sh[];
    const int b = blockIdx.y, y0 = blockIdx.x * band, r = t.r, rows = band + 2 * r;
    float *raw = sh;               // rows y0 - r .. y0 + band + r - 1 (zero outside the bitmap)
    float *hor = sh + rows * Wb;   // the same rows blurred along x
    const TexT *src = in + (size_t)b * Hb * Wb;
    for (int i = threadIdx.x; i < rows * Wb; i += 256) {
        const int yy = y0 - r + i / Wb, xx = i - (i / Wb) * Wb;
        raw[i] = (yy >= 0 && yy < Hb) ? texel<TexT>(src[(size_t)yy * Wb + xx]) : 0.f;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < rows * Wb; i += 256) {
        const int yy = i / Wb, xx = i - yy * Wb;
        float acc = 0.f;
        for (int d = -r; d <= r; ++d) {
            const int x2 = xx + d;
            if (x2 >= 0 && x2 < Wb) acc = fmaf(t.w[d + r], raw[yy * Wb + x2], acc);
        }
        hor[i] = acc;
    }
    __syncthreads();
    TexT *dst = out + (size_t)b * Hb * Wb;
    for (int i = threadIdx.x; i < band * Wb; i += 256) {
        const int yl = i / Wb, xx = i - yl * Wb, yy = y0 + yl;
        if (yy >= Hb) continue;
        float acc = 0.f;
        for (int d = -r; d <= r; ++d) acc = fmaf(t.w[d + r], hor[(yl + r + d) * Wb + xx], acc);
        dst[(size_t)yy * Wb + xx] = from_f32<TexT>(acc);
    }
}

// ------------------------------------------------------------------------------------------
// Structure-aware initialisation (Sec. 3.2.2)
// ------------------------------------------------------------------------------------------
constexpr int LV_T = 16;      // output pixels per workgroup edge
constexpr int LV_HMAX = 7;    // largest window half-width (15 x 15)
constexpr int SCAN_ITEMS = 8; // int64 weights per thread of a scan block
constexpr int SCAN_BLOCK = 256 * SCAN_ITEMS;

// Ordering of non-negative doubles = ordering of their bit patterns as unsigned integers.
__device__ __forceinline__ unsigned long long dbits(double x)
{
    return (unsigned long long)__double_as_longlong(x);
}

// LV of a 16 x 16 pixel block: the (16 + 2h)^2 window of the three channels is staged in LDS;
// each lane sums its pixel's window (only pixels inside the image) in float64.
__global__ void __launch_bounds__(256)
k_local_var(const float *__restrict__ img, int H, int W, int h, double *__restrict__ lv,
            unsigned long long *__restrict__ bmm)
{
    constexpr int S = LV_T + 2 * LV_HMAX;
    __shared__ float s[3][S][S];
    const int bx = blockIdx.x * LV_T, by = blockIdx.y * LV_T, e = LV_T + 2 * h;
    const size_t plane = (size_t)H * W;
    for (int i = threadIdx.x; i < 3 * e * e; i += 256) {
        const int c = i / (e * e), q = i - c * e * e, yy = by - h + q / e, xx = bx - h + q % e;
        s[c][q / e][q % e] = (yy >= 0 && yy < H && xx >= 0 && xx < W)
                                 ? img[c * plane + (size_t)yy * W + xx] : 0.f;
    }
    __syncthreads();
    const int lx = threadIdx.x % LV_T, ly = threadIdx.x / LV_T;
    const int x = bx + lx, y = by + ly;
    double v = 0.0;
    const bool ok = x < W && y < H;
    if (ok) {
        const int x0 = max(x - h, 0) - (bx - h), x1 = min(x + h, W - 1) - (bx - h);
        const int y0 = max(y - h, 0) - (by - h), y1 = min(y + h, H - 1) - (by - h);
        const double n = (double)((x1 - x0 + 1) * (y1 - y0 + 1));
        for (int c = 0; c < 3; ++c) {
            double s1 = 0.0, s2 = 0.0;
            for (int yy = y0; yy <= y1; ++yy)
                for (int xx = x0; xx <= x1; ++xx) {
                    const double a = s[c][yy][xx];
                    s1 += a;
                    s2 = fma(a, a, s2);
                }
            const double m = s1 / n;
            v += s2 / n - m * m;
        }
        v = fmax(v / 3.0, 0.0);  // the one-pass form can round a zero variance below zero
        lv[(size_t)y * W + x] = v;
    }
    // the block's min / max of the map (bit patterns of non-negative doubles), written to its
    // own slot (k_lv_minmax reduces the slots: no same-address atomics across the grid)
    unsigned long long lo = ok ? dbits(v) : 0x7ff0000000000000ull, hi = ok ? dbits(v) : 0ull;
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long a = __shfl_xor(lo, o), b = __shfl_xor(hi, o);
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
    }
    __shared__ unsigned long long s_lo[4], s_hi[4];
    if ((threadIdx.x & 63) == 0) {
        s_lo[threadIdx.x >> 6] = lo;
        s_hi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) {
            lo = s_lo[w] < lo ? s_lo[w] : lo;
            hi = s_hi[w] > hi ? s_hi[w] : hi;
        }
        const size_t b = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
        bmm[2 * b] = lo;
        bmm[2 * b + 1] = hi;
    }
}

// The map's min / max from the blocks' slots: one workgroup.
__global__ void __launch_bounds__(1024)
k_lv_minmax(const unsigned long long *__restrict__ bmm, int nblocks,
            unsigned long long *__restrict__ minmax)
{
    unsigned long long lo = 0x7ff0000000000000ull, hi = 0ull;
    for (int b = threadIdx.x; b < nblocks; b += 1024) {
        lo = bmm[2 * b] < lo ? bmm[2 * b] : lo;
        hi = bmm[2 * b + 1] > hi ? bmm[2 * b + 1] : hi;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long a = __shfl_xor(lo, o), b = __shfl_xor(hi, o);
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
    }
    __shared__ unsigned long long s_lo[16], s_hi[16];
    if ((threadIdx.x & 63) == 0) {
        s_lo[threadIdx.x >> 6] = lo;
        s_hi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 16; ++w) {
            lo = s_lo[w] < lo ? s_lo[w] : lo;
            hi = s_hi[w] > hi ? s_hi[w] : hi;
        }
        minmax[0] = lo;
        minmax[1] = hi;
    }
}

// NLV (float32, the caller's map) and the integer sampling weights computed from it.
__global__ void __launch_bounds__(256)
k_nlv(const double *__restrict__ lv, long long n, const unsigned long long *__restrict__ minmax,
      double base, float *__restrict__ nlv_out, long long *__restrict__ w)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double lo = __longlong_as_double((long long)minmax[0]);
    const double hi = __longlong_as_double((long long)minmax[1]);
    const double q = hi > lo ? (lv[i] - lo) / (hi - lo) : 0.0;
    const float nf = (float)q;
    nlv_out[i] = nf;
    const double wd = base + (1.0 - base) * (double)nf;  // built without contraction
    w[i] = (long long)floor(wd * 16777216.0);
}

// Inclusive int64 scan in three launches: per-block scans (2,048 values, 8 per lane) that also
// leave each block's total; a one-workgroup scan of the totals; the offsets added back.
__device__ __forceinline__ long long wave_incl_scan(long long x, int lane)
{
    for (int o = 1; o < 64; o <<= 1) {
        const long long y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

__global__ void __launch_bounds__(256)
k_scan_blocks(long long *__restrict__ w, long long n, long long *__restrict__ bsum)
{
    __shared__ long long wsum[4];
    const long long base = (long long)blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_ITEMS;
    long long v[SCAN_ITEMS];
    long long run = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = base + k < n ? w[base + k] : 0;
        run += v[k];
        v[k] = run;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long long incl = wave_incl_scan(run, lane);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    long long off = incl - run;
    for (int q = 0; q < wave; ++q) off += wsum[q];
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k)
        if (base + k < n) w[base + k] = v[k] + off;
    if (threadIdx.x == 255) bsum[blockIdx.x] = off + run;
}

__global__ void __launch_bounds__(1024) k_scan_sums(long long *__restrict__ bsum, int nb)
{
    __shared__ long long wsum[16];
    __shared__ long long carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int b0 = 0; b0 < nb; b0 += 1024) {
        const int i = b0 + threadIdx.x;
        const long long x = i < nb ? bsum[i] : 0;
        const long long incl = wave_incl_scan(x, lane);
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        long long off = carry;
        for (int q = 0; q < wave; ++q) off += wsum[q];
        if (i < nb) bsum[i] = incl + off;
        __syncthreads();
        if (threadIdx.x == 1023) carry = incl + off;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256)
k_scan_add(long long *__restrict__ w, long long n, const long long *__restrict__ bsum)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n && i >= SCAN_BLOCK) w[i] += bsum[i / SCAN_BLOCK - 1];
}

// One primitive per lane: inverse-CDF draw of its pixel, then its parameter row.
__global__ void __launch_bounds__(256)
k_sa_sample(const long long *__restrict__ cdf, long long n, const float *__restrict__ nlv,
            const float *__restrict__ img, int H, int W, const float *__restrict__ u_pos,
            const float *__restrict__ u_theta, const float *__restrict__ z, int N, double s_min,
            double s_max, double nu_init, double sigma_c, float *__restrict__ params)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const long long total = cdf[n - 1];
    long long t = (long long)floor((double)u_pos[i] * (double)total);
    if (t >= total) t = total - 1;
    long long lo = 0, hi = n - 1;  // first p with cdf[p] > t
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if (cdf[mid] > t) hi = mid; else lo = mid + 1;
    }
    const int p = (int)lo, x = p % W, y = p / W;
    const double s = s_max - (s_max - s_min) * (double)nlv[p];
    float *row = params + (size_t)i * 8;
    row[0] = (float)x;
    row[1] = (float)y;
    row[2] = (float)log(s);
    row[3] = (float)(2.0 * M_PI * (double)u_theta[i]);
    row[4] = (float)nu_init;
    const size_t plane = (size_t)H * W;
    for (int c = 0; c < 3; ++c) {
        double v = (double)img[c * plane + p] + sigma_c * (double)z[(size_t)i * 3 + c];
        v = fmin(fmax(v, 1e-3), 1.0 - 1e-3);
        row[5 + c] = (float)log(v / (1.0 - v));
    }
}

// ------------------------------------------------------------------------------------------
// Noise canvas (Eq. 8): Philox4x64-10, one block per pixel
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(unsigned long long (&c)[4], unsigned long long k0,
                                              unsigned long long k1)
{
    const unsigned long long M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const unsigned long long W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const unsigned long long hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const unsigned long long hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const unsigned long long n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += W0;
        k1 += W1;
    }
}

__global__ void __launch_bounds__(256)
k_noise(unsigned long long seed, unsigned long long iter, long long npix,
        float *__restrict__ bg)
{
    const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
    if (p >= npix) return;
    unsigned long long c[4] = {(unsigned long long)p, iter, 0ull, 0ull};
    philox4x64_10(c, seed, 0ull);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) bg[ch * npix + p] = (float)(c[ch] >> 40) * 0x1p-24f;
}

// ------------------------------------------------------------------------------------------
// Spatial-constraint loss (Eq. 9) and re-initialisation (Supp. Sec. S1.4.2)
// ------------------------------------------------------------------------------------------
// A grid of at most CONSTRAINT_BLOCKS workgroups strides over the pixels; each workgroup adds
// its share of the loss with one atomic (a wave-level atomic per 64 pixels on one address
// serialised: 0.83 ms at 2048^2).
constexpr int CONSTRAINT_BLOCKS = 2048;

__global__ void __launch_bounds__(256)
k_constraint(const float *__restrict__ I, const float *__restrict__ A,
             const float *__restrict__ t, const float *__restrict__ ta, long long npix,
             float lam, float *__restrict__ gI, float *__restrict__ gA, float *__restrict__ loss)
{
    float acc = 0.f;
    const float inv3 = 1.f / (3.f * (float)npix), inv1 = 1.f / (float)npix;
    for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < npix;
         p += (long long)gridDim.x * 256) {
        const bool m = ta[p] > 0.f;
        for (int c = 0; c < 3; ++c) {
            const float d = m ? I[c * npix + p] - t[c * npix + p] : 0.f;
            gI[c * npix + p] = 2.f * d * inv3;
            acc = fmaf(d * d, inv3, acc);
        }
        const float e = A[p] - ta[p];
        gA[p] = 2.f * lam * e * inv1;
        acc = fmaf(lam * e * e, inv1, acc);
    }
    if (!loss) return;
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    __shared__ float s_acc[4];
    if ((threadIdx.x & 63) == 0) s_acc[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float tot = s_acc[0] + s_acc[1] + s_acc[2] + s_acc[3];
        if (tot != 0.f) atomicAdd(loss, tot);
    }
}

__global__ void __launch_bounds__(256)
k_reinit(float *__restrict__ params, float *__restrict__ m, float *__restrict__ v,
         const float *__restrict__ prop, int N, double logit_thr, int *__restrict__ count)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= N || !((double)params[(size_t)i * 8 + 4] < logit_thr)) return;
    for (int q = 0; q < 8; ++q) {
        params[(size_t)i * 8 + q] = prop[(size_t)i * 8 + q];
        if (m) m[(size_t)i * 8 + q] = 0.f;
        if (v) v[(size_t)i * 8 + q] = 0.f;
    }
    if (count) atomicAdd(count, 1);
}

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

struct SaLayout {
    size_t minmax, bmm, lv, cdf, bsum, total;
};

SaLayout sa_layout(long long npix, int H, int W)
{
    SaLayout L;
    const long long nb = (npix + SCAN_BLOCK - 1) / SCAN_BLOCK;
    const long long nblk = (long long)((W + LV_T - 1) / LV_T) * ((H + LV_T - 1) / LV_T);
    L.minmax = 0;
    L.bmm = up256(16);
    L.lv = L.bmm + up256(16 * (size_t)nblk);
    L.cdf = L.lv + up256(8 * (size_t)npix);
    L.bsum = L.cdf + up256(8 * (size_t)npix);
    L.total = L.bsum + up256(8 * (size_t)nb);
    return L;
}

int launched() { return hipGetLastError() == hipSuccess ? DBMP_OK : DBMP_EHIP; }

}  // namespace
}  // namespace dbmp

using namespace dbmp;

extern "C" {

int dbmp_blur_atlas(dbmp_aids_stream stream, const void *atlas, int B, int Hb, int Wb,
                    int atlas_dtype, float sigma, float truncate, void *out)
{
    if (!atlas || !out || B < 1 || Hb < 1 || Wb < 1 || Wb > 1024) return DBMP_EINVAL;
    if (atlas_dtype != DBMP_F32 && atlas_dtype != DBMP_BF16 && atlas_dtype != DBMP_F16)
        return DBMP_EINVAL;
    if (!(sigma > 0.f && sigma <= 8.f) || !(truncate > 0.f)) return DBMP_EINVAL;
    const int r = (int)(truncate * (double)sigma + 0.5);
    if (r > BLUR_RMAX) return DBMP_EINVAL;
    const size_t esz = atlas_dtype == DBMP_F32 ? 4 : 2;
    const char *a = (const char *)atlas, *o = (const char *)out;
    const size_t bytes = esz * (size_t)B * Hb * Wb;
    if (a < o + bytes && o < a + bytes) return DBMP_EINVAL;  // overlapping buffers
    BlurTaps t{};
    t.r = r;
    double w[2 * BLUR_RMAX + 1], sum = 0.0;
    for (int d = -r; d <= r; ++d) sum += (w[d + r] = exp(-(double)d * d / (2.0 * sigma * sigma)));
    for (int d = -r; d <= r; ++d) t.w[d + r] = (float)(w[d + r] / sum);
    int band = BLUR_LDS_BYTES / (8 * Wb) - 2 * r;
    if (band > 64) band = 64;
    if (band < 1) return DBMP_EINVAL;  // the band does not fit in LDS
    const size_t lds = 8 * (size_t)(band + 2 * r) * Wb;
    const dim3 grid((Hb + band - 1) / band, B);
    hipStream_t st = (hipStream_t)stream;
    if (atlas_dtype == DBMP_F32)
        k_blur<float><<<grid, 256, lds, st>>>((const float *)atlas, (float *)out, Hb, Wb, band, t);
    else if (atlas_dtype == DBMP_F16)
        k_blur<_Float16><<<grid, 256, lds, st>>>((const _Float16 *)atlas, (_Float16 *)out, Hb, Wb,
                                                  band, t);
    else
        k_blur<uint16_t><<<grid, 256, lds, st>>>((const uint16_t *)atlas, (uint16_t *)out, Hb, Wb,
                                                  band, t);
    return launched();
}

long long dbmp_sa_init_workspace_bytes(int H, int W)
{
    if (H < 1 || W < 1 || (long long)H * W >= INT_MAX) return -1;
    return (long long)sa_layout((long long)H * W, H, W).total;
}

int dbmp_sa_init(dbmp_aids_stream stream, const float *target, int H, int W, int win,
                 double base, const float *u_pos, const float *u_theta, const float *z_col, int N,
                 double s_min, double s_max, double nu_init, double sigma_c, void *workspace,
                 long long workspace_bytes, float *nlv_out, float *params_out)
{
    if (!target || !workspace || !nlv_out || H < 1 || W < 1 || N < 0) return DBMP_EINVAL;
    if ((long long)H * W >= INT_MAX) return DBMP_EINVAL;
    if (N > 0 && (!u_pos || !u_theta || !z_col || !params_out)) return DBMP_EINVAL;
    if (win < 1 || win > 2 * LV_HMAX + 1 || !(win & 1)) return DBMP_EINVAL;
    if (!(base >= 0.0 && base <= 1.0) || !(s_min > 0.0) || !(s_max >= s_min)) return DBMP_EINVAL;
    if (!(sigma_c >= 0.0) || ((uintptr_t)workspace & 15)) return DBMP_EINVAL;
    const long long npix = (long long)H * W;
    const SaLayout L = sa_layout(npix, H, W);
    if (workspace_bytes < (long long)L.total) return DBMP_EINVAL;
    char *ws = (char *)workspace;
    auto *minmax = (unsigned long long *)(ws + L.minmax);
    auto *bmm = (unsigned long long *)(ws + L.bmm);
    auto *lv = (double *)(ws + L.lv);
    auto *cdf = (long long *)(ws + L.cdf);
    auto *bsum = (long long *)(ws + L.bsum);
    hipStream_t st = (hipStream_t)stream;
    const dim3 lvg((W + LV_T - 1) / LV_T, (H + LV_T - 1) / LV_T);
    k_local_var<<<lvg, 256, 0, st>>>(target, H, W, win / 2, lv, bmm);
    k_lv_minmax<<<1, 1024, 0, st>>>(bmm, (int)(lvg.x * lvg.y), minmax);
    const unsigned g = (unsigned)((npix + 255) / 256);
    k_nlv<<<g, 256, 0, st>>>(lv, npix, minmax, base, nlv_out, cdf);
    const int nb = (int)((npix + SCAN_BLOCK - 1) / SCAN_BLOCK);
    k_scan_blocks<<<nb, 256, 0, st>>>(cdf, npix, bsum);
    if (nb > 1) {
        k_scan_sums<<<1, 1024, 0, st>>>(bsum, nb);
        k_scan_add<<<g, 256, 0, st>>>(cdf, npix, bsum);
    }
    if (N > 0)
        k_sa_sample<<<(N + 255) / 256, 256, 0, st>>>(cdf, npix, nlv_out, target, H, W, u_pos,
                                                     u_theta, z_col, N, s_min, s_max, nu_init,
                                                     sigma_c, params_out);
    return launched();
}

int dbmp_noise_canvas(dbmp_aids_stream stream, unsigned long long seed,
                      unsigned long long iteration, int H, int W, float *bg_out)
{
    if (!bg_out || H < 1 || W < 1 || (long long)H * W >= INT_MAX) return DBMP_EINVAL;
    const long long npix = (long long)H * W;
    k_noise<<<(unsigned)((npix + 255) / 256), 256, 0, (hipStream_t)stream>>>(seed, iteration,
                                                                               npix, bg_out);
    return launched();
}

int dbmp_constraint_loss(dbmp_aids_stream stream, const float *image, const float *alpha,
                         const float *target, const float *target_alpha, int H, int W,
                         float lambda, float *dL_dimage, float *dL_dalpha, float *loss)
{
    if (!image || !alpha || !target || !target_alpha || !dL_dimage || !dL_dalpha) return DBMP_EINVAL;
    if (H < 1 || W < 1 || (long long)H * W >= INT_MAX || !(lambda >= 0.f)) return DBMP_EINVAL;
    const long long npix = (long long)H * W;
    const long long blocks = std::min<long long>((npix + 255) / 256, CONSTRAINT_BLOCKS);
    k_constraint<<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>(
        image, alpha, target, target_alpha, npix, lambda, dL_dimage, dL_dalpha, loss);
    return launched();
}

int dbmp_reinit_transparent(dbmp_aids_stream stream, float *params, float *m, float *v,
                            const float *proposal, int N, double threshold, int32_t *count)
{
    if (N < 0 || (N > 0 && (!params || !proposal))) return DBMP_EINVAL;
    if (!(threshold > 0.0 && threshold < 1.0)) return DBMP_EINVAL;
    if (N == 0) return DBMP_OK;
    const double thr = threshold;
    k_reinit<<<(N + 255) / 256, 256, 0, (hipStream_t)stream>>>(params, m, v, proposal, N,
                                                              log(thr / (1.0 - thr)), count);
    return launched();
}

}  // extern "C"
