// Kernels of the learned initialiser: a small CNN (3x3 stride-2 convolutions, then a two-layer
// MLP head) that maps a target image to primitive parameters. Training and inference run here,
// in bfloat16 with float32 accumulation on the matrix cores of gfx950 (v_mfma_f32_16x16x32_bf16).
//
// Every layer is one matrix product C[M][N] = sum_k A(m, k) B(k, n), computed by one tiled
// kernel whose operands are produced by gather functors:
//   convolution forward      M = output pixels (b, oy, ox), N = out channels, K = (ky, kx, ic):
//                            A = the image patch under the filter (implicit im2col), B = W;
//   convolution grad-input   one product per parity class of input pixels (y % 2, x % 2):
//                            M = the class's pixels, N = in channels, K = (its taps, oc):
//                            A = output gradients that reach (y, x) through those taps,
//                            B = W with (ic) and (oc) swapped (a transposed copy);
//   convolution grad-weight  M = out channels, N = (ky, kx, ic), K = output pixels:
//                            A = output gradients, B = image patches (both read across K);
//   dense layers             the same three with plain row-major operands.
// Activations are NHWC bfloat16 (a channel run of 8 is one 16-byte load), weights are
// [out][ky][kx][in]; the first layer's 3 input channels are zero-padded to 8.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "dbmp_cnn.h"

namespace dbmp_cnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16;

// float -> bfloat16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ u16 f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}
__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float((uint32_t)h << 16); }

// ------------------------------------------------------------------------------------------
// Tiled product: 64 x 64 output tile per 256-thread workgroup, K in steps of 64. Each wave
// computes a 32 x 32 quarter as 2 x 2 MFMA tiles of 16 x 16 (two 16x16x32 MFMAs per tile and
// K step). Operand tiles are staged in LDS with K contiguous (row pitch 72 bf16), so every
// lane's 8-element MFMA operand is one 16-byte LDS read. Every thread loads KS = 2 chunks of
// 8 elements per operand and step (one per 32-wide half of the step); the loads for the next
// step are issued before the MFMAs of the current one.
// ------------------------------------------------------------------------------------------
constexpr int BM = 64, BN = 64, BK = 64, KS = BK / 32, NT = 256, LDK = BK + 8;

// Operand loaders, by how their elements lie in memory:
//   VEC   elements (row, k .. k+7) are contiguous: one 16-byte load (thread t loads row t/4,
//         k chunk (t%4)*8);
//   TVEC  elements (row .. row+7, k) are contiguous (an operand read across K whose rows run
//         along memory, e.g. NHWC channels): one 16-byte load (thread t loads k t/8, row chunk
//         (t%8)*8), written into the K-contiguous LDS tile transposed, 8 two-byte stores;
//   SCAL  8 scalar loads along K (thread t loads row t%64, k chunk (t/64)*8, so a wave reads 64
//         consecutive rows): the fallback for row counts or pitches that are not multiples of 8.
enum { SCAL = 0, VEC = 1, TVEC = 2 };

struct LPlain {  // element (row, k) = p[row * ld + k]
    static constexpr int KIND = VEC;
    const u16 *p;
    int ld, R, K;
    __device__ uint4 load8(int row, int k) const
    {
        if (row >= R || k >= K) return make_uint4(0, 0, 0, 0);
        return *reinterpret_cast<const uint4 *>(p + (size_t)row * ld + k);
    }
};

template <int KD>
struct LTrans {  // element (row, k) = p[k * ld + row]; TVEC needs ld % 8 == 0
    static constexpr int KIND = KD;
    const u16 *p;
    int ld, R, K;
    __device__ uint4 load8t(int row, int k) const  // rows row .. row+7 at k (row % 8 == 0)
    {
        if (k >= K || row >= R) return make_uint4(0, 0, 0, 0);
        if (row + 8 <= R) return *reinterpret_cast<const uint4 *>(p + (size_t)k * ld + row);
        u16 e[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) e[i] = row + i < R ? p[(size_t)k * ld + row + i] : 0;
        return make_uint4(e[0] | ((uint32_t)e[1] << 16), e[2] | ((uint32_t)e[3] << 16),
                          e[4] | ((uint32_t)e[5] << 16), e[6] | ((uint32_t)e[7] << 16));
    }
    __device__ u16 load1(int row, int k) const
    {
        if (row >= R || k >= K) return 0;
        return p[(size_t)k * ld + row];
    }
};

struct LIm2col {  // row = output pixel (b, oy, ox), k = (ky, kx, ic); x NHWC [B][H][W][C]
    static constexpr int KIND = VEC;
    const u16 *x;
    int H, W, C, OH, OW, M, K;
    __device__ uint4 load8(int m, int k) const
    {
        if (m >= M || k >= K) return make_uint4(0, 0, 0, 0);
        const int tap = k / C, ic = k - tap * C;
        const int ky = tap / 3, kx = tap - 3 * ky;
        const int b = m / (OH * OW), r = m - b * OH * OW;
        const int oy = r / OW, ox = r - oy * OW;
        const int iy = 2 * oy + ky - 1, ix = 2 * ox + kx - 1;
        if (iy < 0 || iy >= H || ix < 0 || ix >= W) return make_uint4(0, 0, 0, 0);
        return *reinterpret_cast<const uint4 *>(x + (((size_t)b * H + iy) * W + ix) * C + ic);
    }
};

template <int KD>
struct LIm2colT {  // row = (ky, kx, ic), k = output pixel (b, oy, ox); x NHWC [B][H][W][C]
    static constexpr int KIND = KD;  // TVEC needs C % 8 == 0 (8 rows share one tap)
    const u16 *x;
    int H, W, C, OH, OW, R, K;
    __device__ uint4 load8t(int n, int k) const  // rows n .. n+7 at k (n % 8 == 0)
    {
        if (n >= R || k >= K) return make_uint4(0, 0, 0, 0);
        const int tap = n / C, ic = n - tap * C;
        const int ky = tap / 3, kx = tap - 3 * ky;
        const int b = k / (OH * OW), r = k - b * OH * OW;
        const int oy = r / OW, ox = r - oy * OW;
        const int iy = 2 * oy + ky - 1, ix = 2 * ox + kx - 1;
        if (iy < 0 || iy >= H || ix < 0 || ix >= W) return make_uint4(0, 0, 0, 0);
        return *reinterpret_cast<const uint4 *>(x + (((size_t)b * H + iy) * W + ix) * C + ic);
    }
    __device__ u16 load1(int n, int k) const
    {
        if (n >= R || k >= K) return 0;
        const int tap = n / C, ic = n - tap * C;
        const int ky = tap / 3, kx = tap - 3 * ky;
        const int b = k / (OH * OW), r = k - b * OH * OW;
        const int oy = r / OW, ox = r - oy * OW;
        const int iy = 2 * oy + ky - 1, ix = 2 * ox + kx - 1;
        if (iy < 0 || iy >= H || ix < 0 || ix >= W) return 0;
        return x[(((size_t)b * H + iy) * W + ix) * C + ic];
    }
};

// Epilogues: called once per output element inside the tile bounds.
struct EAct {  // out = act(acc + bias[n]) as bf16 (and optionally float32), row pitch ld
    const float *bias;
    int relu;
    u16 *out;
    float *out32;
    int ld;
    __device__ void operator()(int m, int n, float v) const
    {
        if (bias) v += bias[n];
        if (relu) v = fmaxf(v, 0.f);
        const size_t i = (size_t)m * ld + n;
        if (out) out[i] = f2bf(v);
        if (out32) out32[i] = v;
    }
};

// The input gradient of a stride-2 convolution, one parity class of input pixels at a time: a
// pixel (y, x) with y % 2 == py, x % 2 == px is reached only by the taps with ky = (y + 1) % 2
// (mod 2) and kx likewise (1 tap, 2 or 4: ky = ky0 + 2 i, i < nky), so each class is a product
// over those taps alone, a quarter of the work of running all 9 taps over every pixel.
struct Phase {
    int py, px;     // the class's pixel parities
    int ky0, nky;   // its taps along y: ky0, ky0 + 2, ... (nky of them)
    int kx0, nkx;
};
// class z = 2 py + px: y even is reached by ky = 1 alone, y odd by ky = 0 and 2 (likewise x)
__device__ __forceinline__ Phase phase_of(int z)
{
    const int py = z >> 1, px = z & 1;
    return Phase{py, px, py ? 0 : 1, py ? 2 : 1, px ? 0 : 1, px ? 2 : 1};
}

struct LCol2imPhase {  // row = pixel (b, hy, hx) of the class, k = (tap, oc); dz NHWC
    static constexpr int KIND = VEC;
    const u16 *dz;
    int H, W, Co, OH, OW, M, K;
    Phase ph;
    __device__ uint4 load8(int m, int k) const
    {
        if (m >= M || k >= K) return make_uint4(0, 0, 0, 0);
        const int t = k / Co, oc = k - t * Co;
        const int ty = t / ph.nkx, tx = t - ty * ph.nkx;
        const int ky = ph.ky0 + 2 * ty, kx = ph.kx0 + 2 * tx;
        const int W2 = W >> 1, HW4 = (H >> 1) * W2;
        const int b = m / HW4, r = m - b * HW4, hy = r / W2, hx = r - hy * W2;
        const int ty2 = 2 * hy + ph.py + 1 - ky, tx2 = 2 * hx + ph.px + 1 - kx;  // = 2 oy, 2 ox
        if (ty2 < 0 || tx2 < 0) return make_uint4(0, 0, 0, 0);
        const int oy = ty2 >> 1, ox = tx2 >> 1;
        if (oy >= OH || ox >= OW) return make_uint4(0, 0, 0, 0);
        return *reinterpret_cast<const uint4 *>(dz + (((size_t)b * OH + oy) * OW + ox) * Co + oc);
    }
};

struct LTapW {  // row = ic, k = (tap of the class, oc); wt [Cin][3][3][Cout]
    static constexpr int KIND = VEC;
    const u16 *w;
    int R, Co, K;
    Phase ph;
    __device__ uint4 load8(int row, int k) const
    {
        if (row >= R || k >= K) return make_uint4(0, 0, 0, 0);
        const int t = k / Co, oc = k - t * Co;
        const int ty = t / ph.nkx, tx = t - ty * ph.nkx;
        const int ky = ph.ky0 + 2 * ty, kx = ph.kx0 + 2 * tx;
        return *reinterpret_cast<const uint4 *>(w + ((size_t)(row * 3 + ky) * 3 + kx) * Co + oc);
    }
};

struct EMaskPhase {  // EMask for row m of a parity class: the pixel it stands for
    const u16 *mask;
    u16 *out;
    int C, H, W;
    Phase ph;
    __device__ void operator()(int m, int n, float v) const
    {
        const int W2 = W >> 1, HW4 = (H >> 1) * W2;
        const int b = m / HW4, r = m - b * HW4, hy = r / W2, hx = r - hy * W2;
        const size_t i = (((size_t)b * H + 2 * hy + ph.py) * W + 2 * hx + ph.px) * C + n;
        if (mask && !(bf2f(mask[i]) > 0.f)) v = 0.f;
        out[i] = f2bf(v);
    }
};

struct EMask {  // out = acc * [mask > 0] as bf16: the gradient through the producing ReLU
    const u16 *mask;
    u16 *out;
    int ld;
    __device__ void operator()(int m, int n, float v) const
    {
        const size_t i = (size_t)m * ld + n;
        if (mask && !(bf2f(mask[i]) > 0.f)) v = 0.f;
        out[i] = f2bf(v);
    }
};

// The four parity classes run as one launch (gridDim.z = 4, no split of K): a workgroup takes
// its class from blockIdx.z and sets its operands' taps and K from it.
template <class L>
struct is_phased {
    static constexpr bool value = false;
};
template <>
struct is_phased<LCol2imPhase> {
    static constexpr bool value = true;
};

struct EAdd {  // out += acc (float atomics: split-K partial sums)
    float *out;
    int ld;
    __device__ void operator()(int m, int n, float v) const
    {
        unsafeAtomicAdd(out + (size_t)m * ld + n, v);
    }
};

template <class L>
__device__ __forceinline__ void fetch(const L &l, int row0, int k0, uint4 &v)
{
    if constexpr (L::KIND == VEC) {
        v = l.load8(row0 + (int)(threadIdx.x >> 2), k0 + (int)(threadIdx.x & 3) * 8);
    } else if constexpr (L::KIND == TVEC) {
        v = l.load8t(row0 + (int)(threadIdx.x & 7) * 8, k0 + (int)(threadIdx.x >> 3));
    } else {
        const int row = row0 + (int)(threadIdx.x & 63), k = k0 + (int)(threadIdx.x >> 6) * 8;
        u16 e[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) e[i] = l.load1(row, k + i);
        v.x = e[0] | ((uint32_t)e[1] << 16);
        v.y = e[2] | ((uint32_t)e[3] << 16);
        v.z = e[4] | ((uint32_t)e[5] << 16);
        v.w = e[6] | ((uint32_t)e[7] << 16);
    }
}

template <class L>
__device__ __forceinline__ void stash(u16 *s, const uint4 &v, int koff)
{
    int row, kc;
    if constexpr (L::KIND == TVEC) {  // 8 rows at one k: transposed into the K-contiguous tile
        row = (threadIdx.x & 7) * 8;
        kc = koff + (int)(threadIdx.x >> 3);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 8; ++j)
            s[(row + j) * LDK + kc] = (u16)(w[j >> 1] >> ((j & 1) * 16));
        return;
    }
    if constexpr (L::KIND == VEC) {
        row = threadIdx.x >> 2;
        kc = (threadIdx.x & 3) * 8;
    } else {
        row = threadIdx.x & 63;
        kc = (threadIdx.x >> 6) * 8;
    }
    *reinterpret_cast<uint4 *>(s + row * LDK + koff + kc) = v;
}

// gridDim = (ceil(M / 64), ceil(N / 64), splits): the long dimension (output pixels) on x;
// split z covers K [z * kper, (z + 1) * kper).
template <class LA, class LB, class EP>
__global__ void __launch_bounds__(NT) k_gemm(LA la, LB lb, EP ep, int M, int N, int K, int kper)
{
    __shared__ __attribute__((aligned(16))) u16 sA[BM * LDK];
    __shared__ __attribute__((aligned(16))) u16 sB[BN * LDK];
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    int kbeg = blockIdx.z * kper;
    int kend = min(K, kbeg + kper);
    if constexpr (is_phased<LA>::value) {
        const Phase ph = phase_of(blockIdx.z);
        la.ph = ph;
        lb.ph = ph;
        ep.ph = ph;
        la.K = lb.K = ph.nky * ph.nkx * la.Co;
        kbeg = 0;
        kend = la.K;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int r = lane & 15, kb = (lane >> 4) * 8;
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    uint4 va[KS], vb[KS];
    if (kbeg < kend) {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            fetch(la, m0, kbeg + 32 * s, va[s]);
            fetch(lb, n0, kbeg + 32 * s, vb[s]);
        }
    }
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        __syncthreads();  // the previous step's LDS reads are done
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            stash<LA>(sA, va[s], 32 * s);
            stash<LB>(sB, vb[s], 32 * s);
        }
        __syncthreads();
        if (k0 + BK < kend) {  // next step's operands, in flight during the MFMAs
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                fetch(la, m0, k0 + BK + 32 * s, va[s]);
                fetch(lb, n0, k0 + BK + 32 * s, vb[s]);
            }
        }
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                a[i] = *reinterpret_cast<const bf16x8 *>(sA + (wm * 32 + i * 16 + r) * LDK +
                                                         32 * s + kb);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                b[j] = *reinterpret_cast<const bf16x8 *>(sB + (wn * 32 + j * 16 + r) * LDK +
                                                         32 * s + kb);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] =
                        __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
    // acc[i][j][e] holds C[row][col] with row = (lane / 16) * 4 + e, col = lane % 16 of the
    // 16 x 16 tile (i, j) of this wave's quarter.
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + wm * 32 + i * 16 + (lane >> 4) * 4 + e;
                const int n = n0 + wn * 32 + j * 16 + r;
                if (m < M && n < N) ep(m, n, acc[i][j][e]);
            }
}

template <class LA, class LB, class EP>
static hipError_t gemm(hipStream_t st, const LA &la, const LB &lb, const EP &ep, int M, int N,
                       int K, int splits)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    const int ksteps = (K + BK - 1) / BK;
    splits = std::max(1, std::min(splits, ksteps));
    const int kper = ((ksteps + splits - 1) / splits) * BK;
    splits = (K + kper - 1) / kper;
    dim3 grid((M + BM - 1) / BM, (N + BN - 1) / BN, std::max(splits, 1));
    k_gemm<LA, LB, EP><<<grid, NT, 0, st>>>(la, lb, ep, M, N, K, kper);
    return hipGetLastError();
}

// Splits of a long K so that the grid has about 1,024 workgroups.
static int splits_for(int M, int N, int K)
{
    const long long tiles = (long long)((M + BM - 1) / BM) * ((N + BN - 1) / BN);
    const long long want = std::max(1LL, 1024 / std::max(1LL, tiles));
    const long long ksteps = (K + BK - 1) / BK;
    return (int)std::min(want, std::max(1LL, ksteps / 4));  // >= 256 of K per split
}

// ------------------------------------------------------------------------------------------
// Elementwise kernels
// ------------------------------------------------------------------------------------------
// Column sums of a bf16 matrix [M][N] added into out[N] (bias gradients), N % 8 == 0 and
// N <= 2048: with G = N / 8 column groups, thread t reads the 8 columns of group t % G (one
// 16-byte load) in every (256 / G)-th row of the workgroup's rows; the partial sums meet in LDS
// and each column gets one float atomic per workgroup.
__global__ void __launch_bounds__(256) k_colsum8(const u16 *__restrict__ z, int M, int N,
                                                 int rows_per_block, float *__restrict__ out)
{
    const int G = N >> 3, per = 256 / G;
    const int t = threadIdx.x, g = t % G, ph = t / G;
    const int r0 = blockIdx.x * rows_per_block, r1 = min(M, r0 + rows_per_block);
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    constexpr int U = 4;  // rows in flight per thread
    if (ph < per)
        for (int m0 = r0 + ph; m0 < r1; m0 += U * per) {
            uint4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int m = m0 + u * per;
                v[u] = m < r1 ? *reinterpret_cast<const uint4 *>(z + (size_t)m * N + g * 8)
                              : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t w[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    acc[j] += bf2f((u16)(w[j >> 1] >> ((j & 1) * 16)));
            }
        }
    __shared__ float part[256 * 8];
#pragma unroll
    for (int j = 0; j < 8; ++j) part[t * 8 + j] = acc[j];
    __syncthreads();
    for (int c = t; c < N; c += 256) {
        const int gc = c >> 3, j = c & 7;
        float v = 0.f;
        for (int q = 0; q < per; ++q) v += part[(q * G + gc) * 8 + j];
        unsafeAtomicAdd(out + c, v);
    }
}

// Column sums of a bf16 matrix [M][N] added into out[N] (bias gradients), any N.
__global__ void __launch_bounds__(256) k_colsum(const u16 *__restrict__ z, int M, int N,
                                                int rows_per_block, float *__restrict__ out)
{
    const int n = blockIdx.x * 64 + (threadIdx.x & 63);
    const int q = threadIdx.x >> 6;
    const int r0 = blockIdx.y * rows_per_block;
    const int r1 = min(M, r0 + rows_per_block);
    float s = 0.f;
    if (n < N)
        for (int m = r0 + q; m < r1; m += 4) s += bf2f(z[(size_t)m * N + n]);
    __shared__ float part[256];
    part[threadIdx.x] = s;
    __syncthreads();
    if (q == 0 && n < N) {
        s = part[threadIdx.x] + part[threadIdx.x + 64] + part[threadIdx.x + 128] +
            part[threadIdx.x + 192];
        unsafeAtomicAdd(out + n, s);
    }
}

// Bias gradient: column sums of dz [M][N] added into db (the vector form where it applies).
static hipError_t colsum(hipStream_t st, const u16 *dz, int M, int N, float *db)
{
    if (N % 8 == 0 && N <= 2048 && ((uintptr_t)dz & 15) == 0) {
        const int rows = 2048;
        k_colsum8<<<(M + rows - 1) / rows, 256, 0, st>>>(dz, M, N, rows, db);
    } else {
        const int rows = 4096;
        dim3 grid((N + 63) / 64, (M + rows - 1) / rows);
        k_colsum<<<grid, 256, 0, st>>>(dz, M, N, rows, db);
    }
    return hipGetLastError();
}

// float32 weights [R][T][C] -> bf16 copies in [R][T][C] and transposed [C][T][R] layouts.
__global__ void k_cast(const float *__restrict__ w, int R, int T, int C, u16 *__restrict__ wb,
                       u16 *__restrict__ wt)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)R * T * C;
    if (i >= n) return;
    const int c = (int)(i % C);
    const int t = (int)((i / C) % T);
    const int r = (int)(i / ((long long)C * T));
    const u16 h = f2bf(w[i]);
    if (wb) wb[i] = h;
    if (wt) wt[((size_t)c * T + t) * R + r] = h;
}

// float32 images [B][3][H][W] -> bf16 NHWC [B][H][W][8] (channels 3..7 zero).
__global__ void k_pack(const float *__restrict__ img, int B, int H, int W, u16 *__restrict__ x)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long n = (long long)B * H * W;
    if (i >= n) return;
    const long long b = i / ((long long)H * W), p = i - b * H * W;
    const float *src = img + (size_t)b * 3 * H * W + p;
    const size_t plane = (size_t)H * W;
    uint4 v;
    v.x = f2bf(src[0]) | ((uint32_t)f2bf(src[plane]) << 16);
    v.y = f2bf(src[2 * plane]);
    v.z = 0;
    v.w = 0;
    *reinterpret_cast<uint4 *>(x + (size_t)i * 8) = v;
}

// Parameter regression loss over rows of 8 values: weighted squared error per column, except
// the angle column (3), which uses w (1 - cos(pred - target)) so that full turns cost nothing.
// Writes dpred = scale * dL/dpred (+ extra[i] * xs[column], a gradient reaching the codes from
// elsewhere, e.g. through the renderer) as bf16 and adds the weighted loss sum * scale to *loss.
struct Col8 {
    float v[8];
};

__global__ void __launch_bounds__(256) k_param_loss(const float *__restrict__ pred,
                                                    const float *__restrict__ tgt,
                                                    const float *__restrict__ w, long long n,
                                                    float scale, const float *__restrict__ extra,
                                                    Col8 xs, u16 *__restrict__ dpred,
                                                    float *__restrict__ loss)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.f;
    if (i < n) {
        const int q = (int)(i & 7);
        float g = 0.f;
        if (tgt) {
            const float d = pred[i] - tgt[i];
            if (q == 3) {
                float sn, cs;
                __sincosf(d, &sn, &cs);
                l = w[q] * (1.f - cs);
                g = w[q] * sn;
            } else {
                l = w[q] * d * d;
                g = 2.f * w[q] * d;
            }
        }
        g *= scale;
        if (extra) g = fmaf(extra[i], xs.v[q], g);
        dpred[i] = f2bf(g);
    }
    __shared__ float part[256];
    part[threadIdx.x] = l;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) unsafeAtomicAdd(loss, part[0] * scale);
}

// Per-column affine coding of parameter rows (row r is slot r % slots of a grid x grid
// template): decode  p = clip(t) * scale[q] + bias[q] + centre(slot, q),
//          encode  t = clip((p - bias[q] - centre(slot, q)) / scale[q]),
// where centre is the slot's cell centre for x (q = 0) and y (q = 1) and 0 otherwise, and clip
// limits to [-clip, clip] every column but the angle (3). Slots are numbered block by block
// (block x block cells each, row-major inside; blocks row-major over the grid), so that the
// 64 slots one position of the network's last feature map predicts are one 8 x 8 block.
struct Coding {
    Col8 scale, bias;
    int slots, grid, block;
    float cell, clip;
};

__global__ void k_code(const float *__restrict__ in, long long n, Coding c, int decode,
                       float *__restrict__ out)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int q = (int)(i & 7);
    const int slot = (int)((i >> 3) % c.slots);
    const int bb = c.block * c.block, blk = slot / bb, pos = slot - blk * bb;
    const int bpr = c.grid / c.block;
    const int col = (blk % bpr) * c.block + pos % c.block;
    const int row = (blk / bpr) * c.block + pos / c.block;
    const float centre = q == 0 ? (col + 0.5f) * c.cell : (q == 1 ? (row + 0.5f) * c.cell : 0.f);
    const float lim = q == 3 ? 3.0e38f : c.clip;
    if (decode) {
        const float t = fminf(fmaxf(in[i], -lim), lim);
        out[i] = fmaf(t, c.scale.v[q], c.bias.v[q] + centre);
    } else {
        const float t = (in[i] - c.bias.v[q] - centre) / c.scale.v[q];
        out[i] = fminf(fmaxf(t, -lim), lim);
    }
}

}  // namespace dbmp_cnn

using namespace dbmp_cnn;

static int status(hipError_t e) { return e == hipSuccess ? DBMP_CNN_OK : DBMP_CNN_EHIP; }

extern "C" {

int dbmp_cnn_conv_forward(void *stream, const uint16_t *x, int B, int H, int W, int Cin,
                          const uint16_t *w, const float *bias, int Cout, int relu, uint16_t *y,
                          float *y32)
{
    if (!x || !w || (!y && !y32) || B < 1 || H < 2 || W < 2 || (H & 1) || (W & 1) ||
        Cin < 8 || (Cin & 7) || Cout < 1)
        return DBMP_CNN_EINVAL;
    const int OH = H / 2, OW = W / 2, M = B * OH * OW, K = 9 * Cin;
    LIm2col la{x, H, W, Cin, OH, OW, M, K};
    LPlain lb{w, K, Cout, K};
    EAct ep{bias, relu, y, y32, Cout};
    return status(gemm((hipStream_t)stream, la, lb, ep, M, Cout, K, 1));
}

int dbmp_cnn_conv_backward_data(void *stream, const uint16_t *dz, int B, int H, int W, int Cin,
                                const uint16_t *wt, int Cout, const uint16_t *mask,
                                uint16_t *dx)
{
    if (!dz || !wt || !dx || B < 1 || H < 2 || W < 2 || (H & 1) || (W & 1) || Cin < 1 ||
        Cout < 8 || (Cout & 7) || (Cin & 7))
        return DBMP_CNN_EINVAL;
    const int OH = H / 2, OW = W / 2, M4 = B * OH * OW;
    // one launch over the four parity classes (the kernel sets each class's taps and K)
    const Phase none{0, 0, 0, 0, 0, 0};
    LCol2imPhase la{dz, H, W, Cout, OH, OW, M4, 0, none};
    LTapW lb{wt, Cin, Cout, 0, none};
    EMaskPhase ep{mask, dx, Cin, H, W, none};
    dim3 grid((M4 + BM - 1) / BM, (Cin + BN - 1) / BN, 4);
    k_gemm<LCol2imPhase, LTapW, EMaskPhase><<<grid, NT, 0, (hipStream_t)stream>>>(la, lb, ep, M4,
                                                                                 Cin, 0, 0);
    return status(hipGetLastError());
}

int dbmp_cnn_conv_backward_weight(void *stream, const uint16_t *x, const uint16_t *dz, int B,
                                  int H, int W, int Cin, int Cout, float *dw, float *db)
{
    if (!x || !dz || !dw || B < 1 || H < 2 || W < 2 || (H & 1) || (W & 1) || Cin < 1 ||
        Cout < 1)
        return DBMP_CNN_EINVAL;
    const int OH = H / 2, OW = W / 2, P = B * OH * OW, N = 9 * Cin;
    EAdd ep{dw, N};
    hipStream_t st = (hipStream_t)stream;
    const int sp = splits_for(Cout, N, P);
    hipError_t e;
    // A(oc, p) = dz[p][oc], B(n, p) = patch value: both read across K = output pixels, their
    // rows (channels) contiguous in NHWC, so 16-byte loads where the channel counts allow
    if (Cout % 8 == 0 && Cin % 8 == 0 && ((uintptr_t)dz & 15) == 0 && ((uintptr_t)x & 15) == 0)
        e = gemm(st, LTrans<TVEC>{dz, Cout, Cout, P}, LIm2colT<TVEC>{x, H, W, Cin, OH, OW, N, P},
                 ep, Cout, N, P, sp);
    else
        e = gemm(st, LTrans<SCAL>{dz, Cout, Cout, P}, LIm2colT<SCAL>{x, H, W, Cin, OH, OW, N, P},
                 ep, Cout, N, P, sp);
    if (e == hipSuccess && db) e = colsum(st, dz, P, Cout, db);
    return status(e);
}

int dbmp_cnn_linear_forward(void *stream, const uint16_t *x, int B, int K, const uint16_t *w,
                            const float *bias, int N, int relu, uint16_t *y, float *y32)
{
    if (!x || !w || (!y && !y32) || B < 1 || K < 8 || (K & 7) || N < 1) return DBMP_CNN_EINVAL;
    LPlain la{x, K, B, K};
    LPlain lb{w, K, N, K};
    EAct ep{bias, relu, y, y32, N};
    return status(gemm((hipStream_t)stream, la, lb, ep, B, N, K, 1));
}

int dbmp_cnn_linear_backward_data(void *stream, const uint16_t *dz, int B, int N,
                                  const uint16_t *wt, int K, const uint16_t *mask, uint16_t *dx)
{
    if (!dz || !wt || !dx || B < 1 || N < 8 || (N & 7) || K < 1) return DBMP_CNN_EINVAL;
    LPlain la{dz, N, B, N};
    LPlain lb{wt, N, K, N};  // wt [K][N]
    EMask ep{mask, dx, K};
    return status(gemm((hipStream_t)stream, la, lb, ep, B, K, N, 1));
}

int dbmp_cnn_linear_backward_weight(void *stream, const uint16_t *x, const uint16_t *dz, int B,
                                    int K, int N, float *dw, float *db)
{
    if (!x || !dz || !dw || B < 1 || K < 1 || N < 1) return DBMP_CNN_EINVAL;
    EAdd ep{dw, K};
    hipStream_t st = (hipStream_t)stream;
    const int sp = splits_for(N, K, B);
    hipError_t e;
    // A(n, b) = dz[b][n], B(k, b) = x[b][k]
    if (N % 8 == 0 && K % 8 == 0 && ((uintptr_t)dz & 15) == 0 && ((uintptr_t)x & 15) == 0)
        e = gemm(st, LTrans<TVEC>{dz, N, N, B}, LTrans<TVEC>{x, K, K, B}, ep, N, K, B, sp);
    else
        e = gemm(st, LTrans<SCAL>{dz, N, N, B}, LTrans<SCAL>{x, K, K, B}, ep, N, K, B, sp);
    if (e == hipSuccess && db) e = colsum(st, dz, B, N, db);
    return status(e);
}

int dbmp_cnn_cast_weights(void *stream, const float *w, int R, int T, int C, uint16_t *wb,
                          uint16_t *wt)
{
    if (!w || (!wb && !wt) || R < 1 || T < 1 || C < 1) return DBMP_CNN_EINVAL;
    const long long n = (long long)R * T * C;
    k_cast<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(w, R, T, C, wb, wt);
    return status(hipGetLastError());
}

int dbmp_cnn_pack_input(void *stream, const float *img, int B, int H, int W, uint16_t *x)
{
    if (!img || !x || B < 1 || H < 1 || W < 1) return DBMP_CNN_EINVAL;
    const long long n = (long long)B * H * W;
    k_pack<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(img, B, H, W, x);
    return status(hipGetLastError());
}

int dbmp_cnn_param_loss(void *stream, const float *pred, const float *target,
                        const float *weights8, long long n, float scale, const float *extra,
                        const float *extra_scale8, uint16_t *dpred, float *loss)
{
    if (!pred || (target && !weights8) || (extra && !extra_scale8) || !dpred || n < 0 ||
        (n & 7))
        return DBMP_CNN_EINVAL;
    if (n == 0) return DBMP_CNN_OK;
    Col8 xs{};
    if (extra)
        for (int q = 0; q < 8; ++q) xs.v[q] = extra_scale8[q];
    k_param_loss<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(
        pred, target, weights8, n, scale, extra, xs, dpred, loss);
    return status(hipGetLastError());
}

int dbmp_cnn_code_params(void *stream, const float *in, long long n_rows, int slots, int grid,
                         int block, float cell, const float *scale8, const float *bias8,
                         float clip, int decode, float *out)
{
    if (!in || !out || !scale8 || !bias8 || n_rows < 0 || slots < 1 || grid < 1 || block < 1 ||
        grid % block != 0 || !(clip > 0.f))
        return DBMP_CNN_EINVAL;
    for (int q = 0; q < 8; ++q)
        if (scale8[q] == 0.f) return DBMP_CNN_EINVAL;
    if (n_rows == 0) return DBMP_CNN_OK;
    Coding c{};
    for (int q = 0; q < 8; ++q) {
        c.scale.v[q] = scale8[q];
        c.bias.v[q] = bias8[q];
    }
    c.slots = slots;
    c.grid = grid;
    c.block = block;
    c.cell = cell;
    c.clip = clip;
    const long long n = n_rows * 8;
    k_code<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(in, n, c, decode ? 1 : 0,
                                                                        out);
    return status(hipGetLastError());
}

}  // extern "C"
