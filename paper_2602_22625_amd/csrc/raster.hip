// Forward and backward raster kernels (Sec. 3.1.1-3.1.2; Supp. Eqs. S1-S5).
//
// One workgroup per T x T screen tile, one lane per pixel, the tile's wave64s laid out as 8 x 8
// pixel blocks (the most compact footprint, so whole waves skip primitives they do not touch).
// Each wave walks the tile's primitive list; the primitive record is wave-uniform and is read
// through the scalar cache, so the inverse-affine coefficients sit in SGPRs. Texels are fetched
// from the zero-bordered atlas copy (L1/L2): at these workloads a primitive is minified 2-8x,
// so staging its footprint in LDS would move many more texels than the 4 each pixel samples.
//
// Precision: the canvas -> bitmap map is evaluated in float64 (2 FMAs per coordinate; on
// gfx950 a float64 FMA issues at the rate of a non-packed float32 one), so the bilinear weights
// carry float32 precision even at U ~ 128; sampling and compositing are float32.
//
// Forward: front to back, C += T alpha c, T *= (1 - alpha) (Eqs. 4-5), I = C + T b, A = 1 - T.
// It stores no per-layer state; per pixel it keeps the list position K of the last layer in
// front of which T >= TAU, and T_K.
//
// Backward: the list is walked back to front. Transmittance is recovered per layer from the
// pixel's saved (K, T_K): T_j = T_{j+1} / (1 - alpha_j) for j < K (the same float32 factor the
// forward multiplied by, and 1 - alpha_j >= T_{j+1} >= TAU > 0, so no division by zero even at
// alpha = 1); T_j := 0 behind K. With G the composite behind layer j (starting at the
// background) and B the product of (1 - alpha) behind it (starting at 1):
//     dL/dalpha_j = T_j [ g . (c_j - G) + g_A B ]                          (Supp. Eq. S5)
//     dL/dc_j     = g T_j alpha_j c_j (1 - c_j)                            (Supp. Eq. S4)
//     dL/dnu_j    = dL/dalpha_j alpha_max sigma (1 - sigma) M
//     dL/dU', dL/dV' = dL/dalpha_j alpha_max sigma (dM/dU, dM/dV), then through Eq. (1)-(2) to
//     x, y, log s, theta (Eq. 7).
// The 8 per-lane partials are reduced across the wave with a transposed butterfly (after three
// exchange steps each lane carries one of the 8 sums) and added to dL/dparams with one
// float32 atomic per (wave, primitive, parameter).
#include "dbmp_internal.h"

namespace dbmp {

template <int TS>
struct TileGeom {
    int px, py, pix;
    bool valid;
    ImgDev D;
    int b;
};

template <int TS>
__device__ __forceinline__ TileGeom<TS> tile_geom(int tile, const ImgDev *__restrict__ imgs,
                                                  int n_images)
{
    TileGeom<TS> tg;
    tg.b = find_by_tile(imgs, n_images, tile);
    tg.D = imgs[tg.b];
    const int lt = tile - tg.D.tile_off;
    const int tx = lt % tg.D.ntx, ty = lt / tg.D.ntx;
    constexpr int WPR = TS / 8;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    tg.px = tx * TS + (wave % WPR) * 8 + (lane & 7);
    tg.py = ty * TS + (wave / WPR) * 8 + (lane >> 3);
    tg.valid = tg.px < tg.D.W && tg.py < tg.D.H;
    tg.pix = tg.py * tg.D.W + tg.px;
    return tg;
}

// Bilinear sample of the padded bitmap at (U', V') (Supp. Eqs. S1-S3). Returns M and its
// derivatives along U' and V' on the floor cell.
template <typename TexT>
__device__ __forceinline__ void bilinear(const TexT *__restrict__ atlas, int tex, int Wp, double U,
                                         double V, float &M, float &MU, float &MV)
{
    const double fU = floor(U), fV = floor(V);
    const float wu = (float)(U - fU), wv = (float)(V - fV);
    const int iu = (int)fU, iv = (int)fV;
    const TexT *t = atlas + (tex + iv * Wp + iu);
    const float p00 = texel<TexT>(t[0]), p01 = texel<TexT>(t[1]);
    const float p10 = texel<TexT>(t[Wp]), p11 = texel<TexT>(t[Wp + 1]);
    const float d0 = p01 - p00, d1 = p11 - p10;
    const float top = fmaf(wu, d0, p00);
    const float bot = fmaf(wu, d1, p10);
    MV = bot - top;
    M = fmaf(wv, MV, top);
    MU = fmaf(wv, d1 - d0, d0);
}

// Lanes of the wave whose pixel lies in the primitive's support: four float64 compares whose
// lane masks are combined on the scalar unit.
__device__ __forceinline__ uint64_t support_mask(const PrimRec &r, double U, double V,
                                                 uint64_t valid)
{
    return __ballot(U >= r.Ulo) & __ballot(U < r.Uhi) & __ballot(V >= r.Vlo) &
           __ballot(V < r.Vhi) & valid;
}

template <int TS, typename TexT, bool BG_PP>
__global__ void __launch_bounds__(TS * TS)
k_raster_fwd(const PrimRec *__restrict__ recs, const int *__restrict__ pairs,
             const int *__restrict__ tile_start, const int *__restrict__ tile_count,
             const ImgDev *__restrict__ imgs, int n_images, int n_tiles,
             const TexT *__restrict__ atlas, int Wp, const float *__restrict__ bg,
             float *__restrict__ image, float *__restrict__ alpha, int *__restrict__ saveK,
             float *__restrict__ saveT, const int *__restrict__ flags,
             unsigned long long *__restrict__ pair_counter)
{
    if (flags[F_OVERFLOW]) return;
    const int tile = xcd_remap(blockIdx.x, n_tiles);
    const TileGeom<TS> tg = tile_geom<TS>(tile, imgs, n_images);
    const double xd = tg.px, yd = tg.py;
    const uint64_t vmask = __ballot(tg.valid);
    const int start = tile_start[tile], n = tile_count[(size_t)tile * CNT_STRIDE];
    float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, TK = 1.f;
    int K = -1;
    unsigned long long npairs = 0;  // wave-uniform count of evaluated (pixel, primitive) pairs
    for (int j = 0; j < n; ++j) {
        const PrimRec &r = recs[pairs[start + j]];
        const double U = fma(r.aU, xd, fma(r.bU, yd, r.eU));
        const double V = fma(r.aV, xd, fma(r.bV, yd, r.eV));
        const uint64_t m = support_mask(r, U, V, vmask);
        if (m == 0) continue;  // no lane of this wave touches the primitive
        npairs += __popcll(m);
        const bool in = __builtin_amdgcn_inverse_ballot_w64(m);
        if (in) {
            float M, MU, MV;
            bilinear<TexT>(atlas, r.tex, Wp, U, V, M, MU, MV);
            const float a = r.ka * M;  // Eq. (3)
            if (T >= DBMP_TAU) { K = j; TK = T; }
            const float w = T * a;
            C0 = fmaf(w, r.cr, C0);
            C1 = fmaf(w, r.cg, C1);
            C2 = fmaf(w, r.cb, C2);
            T = T * (1.f - a);
        }
    }
    if ((threadIdx.x & 63) == 0 && npairs)  // spread over slots: no single hot address
        atomicAdd(pair_counter + ((blockIdx.x * (TS * TS / 64) + (threadIdx.x >> 6)) &
                                  (DBMP_COUNTER_SLOTS - 1)),
                  npairs);
    if (!tg.valid) return;
    const ImgDev &D = tg.D;
    const size_t plane = (size_t)D.H * D.W;
    float b0, b1, b2;
    if (BG_PP) {
        const float *bp = bg + 3 * D.pix_off + tg.pix;
        b0 = bp[0]; b1 = bp[plane]; b2 = bp[2 * plane];
    } else {
        b0 = bg[3 * tg.b]; b1 = bg[3 * tg.b + 1]; b2 = bg[3 * tg.b + 2];
    }
    float *ip = image + 3 * D.pix_off + tg.pix;
    ip[0] = fmaf(T, b0, C0);
    ip[plane] = fmaf(T, b1, C1);
    ip[2 * plane] = fmaf(T, b2, C2);
    const long long gp = D.pix_off + tg.pix;
    if (alpha) alpha[gp] = 1.f - T;
    saveK[gp] = K;
    saveT[gp] = TK;
}

// Wave-wide sum of 8 values per lane. Three exchange steps (lane bits 5, 4, 3) halve the
// number of live values each time; three more add within groups of 8 lanes. On return lane l
// holds the wave total of value (l >> 3).
__device__ __forceinline__ float reduce8(const float (&v)[8], int lane)
{
    const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8;
    float w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float send = h5 ? v[i] : v[i + 4];
        const float keep = h5 ? v[i + 4] : v[i];
        w[i] = keep + __shfl_xor(send, 32);
    }
    float x[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const float send = h4 ? w[i] : w[i + 2];
        const float keep = h4 ? w[i + 2] : w[i];
        x[i] = keep + __shfl_xor(send, 16);
    }
    float y = (h3 ? x[1] : x[0]) + __shfl_xor(h3 ? x[0] : x[1], 8);
    y += __shfl_xor(y, 4);
    y += __shfl_xor(y, 2);
    y += __shfl_xor(y, 1);
    return y;
}

template <int TS, typename TexT, bool BG_PP, bool HAS_GA>
__global__ void __launch_bounds__(TS * TS)
k_raster_bwd(const PrimRec *__restrict__ recs, const int *__restrict__ pairs,
             const int *__restrict__ tile_start, const int *__restrict__ tile_count,
             const ImgDev *__restrict__ imgs, int n_images, int n_tiles,
             const TexT *__restrict__ atlas, int Wp, const float *__restrict__ bg,
             const int *__restrict__ saveK, const float *__restrict__ saveT,
             const float *__restrict__ gI, const float *__restrict__ gA,
             float *__restrict__ dparams, double cu1, double cv1, float cu_cv, float cv_cu,
             const int *__restrict__ flags)
{
    if (flags[F_OVERFLOW]) return;
    const int tile = xcd_remap(blockIdx.x, n_tiles);
    const TileGeom<TS> tg = tile_geom<TS>(tile, imgs, n_images);
    const int lane = threadIdx.x & 63;
    const ImgDev &D = tg.D;
    const double xd = tg.px, yd = tg.py;
    const uint64_t vmask = __ballot(tg.valid);
    const size_t plane = (size_t)D.H * D.W;
    const long long gp = D.pix_off + tg.pix;
    float g0 = 0.f, g1 = 0.f, g2 = 0.f, ga = 0.f, G0 = 0.f, G1 = 0.f, G2 = 0.f, TK = 0.f;
    int K = -1;
    if (tg.valid) {
        const float *gp3 = gI + 3 * D.pix_off + tg.pix;
        g0 = gp3[0]; g1 = gp3[plane]; g2 = gp3[2 * plane];
        if (HAS_GA) ga = gA[gp];
        if (BG_PP) {
            const float *bp = bg + 3 * D.pix_off + tg.pix;
            G0 = bp[0]; G1 = bp[plane]; G2 = bp[2 * plane];
        } else {
            G0 = bg[3 * tg.b]; G1 = bg[3 * tg.b + 1]; G2 = bg[3 * tg.b + 2];
        }
        K = saveK[gp];
        TK = saveT[gp];
    }
    float Bk = 1.f, Trun = TK;
    const int start = tile_start[tile], n = tile_count[(size_t)tile * CNT_STRIDE];
    for (int j = n - 1; j >= 0; --j) {
        const int g = pairs[start + j];
        const PrimRec &r = recs[g];
        const double U = fma(r.aU, xd, fma(r.bU, yd, r.eU));
        const double V = fma(r.aV, xd, fma(r.bV, yd, r.eV));
        const uint64_t m = support_mask(r, U, V, vmask);
        if (m == 0) continue;  // no lane of this wave touches the primitive
        const bool in = __builtin_amdgcn_inverse_ballot_w64(m);
        float d[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) d[q] = 0.f;
        if (in) {
            float M, MU, MV;
            bilinear<TexT>(atlas, r.tex, Wp, U, V, M, MU, MV);
            const float a = r.ka * M;
            const float m = 1.f - a;
            float Tj = 0.f;
            if (j == K) {
                Tj = TK;
            } else if (j < K) {
                Tj = Trun / m;
            }
            Trun = Tj;
            const float cr = r.cr, cg = r.cg, cb = r.cb;
            float dal = g0 * (cr - G0);
            dal = fmaf(g1, cg - G1, dal);
            dal = fmaf(g2, cb - G2, dal);
            if (HAS_GA) dal = fmaf(ga, Bk, dal);
            dal *= Tj;
            const float ta = Tj * a;
            d[5] = g0 * ta * cr * (1.f - cr);
            d[6] = g1 * ta * cg * (1.f - cg);
            d[7] = g2 * ta * cb * (1.f - cb);
            const float dM = dal * r.ka;
            d[4] = dM * r.omsig * M;
            const float gU = dM * MU, gV = dM * MV;
            const float Ub = (float)(U - cu1), Vb = (float)(V - cv1);
            d[0] = -(gU * r.faU + gV * r.faV);
            d[1] = -(gU * r.fbU + gV * r.fbV);
            d[2] = -(gU * Ub + gV * Vb);
            d[3] = gU * cu_cv * Vb - gV * cv_cu * Ub;
            G0 = fmaf(m, G0, a * cr);
            G1 = fmaf(m, G1, a * cg);
            G2 = fmaf(m, G2, a * cb);
            Bk *= m;
        }
        const float tot = reduce8(d, lane);
        if ((lane & 7) == 0) unsafeAtomicAdd(dparams + (size_t)g * 8 + (lane >> 3), tot);
    }
}

__global__ void k_fill0(float *__restrict__ p, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// ------------------------------------------------------------------------------------------
// Host launchers
// ------------------------------------------------------------------------------------------

template <int TS, typename TexT, bool BGPP>
static void fwd_t(const RasterArgs &a, hipStream_t st)
{
    k_raster_fwd<TS, TexT, BGPP><<<a.n_tiles, TS * TS, 0, st>>>(
        a.recs, a.pairs, a.tile_start, a.tile_count, a.imgs, a.n_images, a.n_tiles,
        (const TexT *)a.atlas_pad, a.Wp, a.bg, a.image, a.alpha, a.saveK, a.saveT, a.flags,
        a.pair_counter);
}

template <int TS, typename TexT, bool BGPP, bool GA>
static void bwd_t(const RasterArgs &a, hipStream_t st)
{
    const double cu = 0.5 * (a.Wb - 1), cv = 0.5 * (a.Hb - 1);
    k_raster_bwd<TS, TexT, BGPP, GA><<<a.n_tiles, TS * TS, 0, st>>>(
        a.recs, a.pairs, a.tile_start, a.tile_count, a.imgs, a.n_images, a.n_tiles,
        (const TexT *)a.atlas_pad, a.Wp, a.bg, a.saveK, a.saveT, a.gI, a.gA, a.dparams, cu + 1.0,
        cv + 1.0, (float)(cu / cv), (float)(cv / cu), a.flags);
}

template <int TS, typename TexT>
static void fwd_d1(const RasterArgs &a, hipStream_t st)
{
    if (a.bg_pp) fwd_t<TS, TexT, true>(a, st); else fwd_t<TS, TexT, false>(a, st);
}
template <int TS>
static void fwd_d0(const RasterArgs &a, hipStream_t st)
{
    if (a.dtype == 0) fwd_d1<TS, float>(a, st); else fwd_d1<TS, uint16_t>(a, st);
}

template <int TS, typename TexT, bool BGPP>
static void bwd_d2(const RasterArgs &a, hipStream_t st)
{
    if (a.gA) bwd_t<TS, TexT, BGPP, true>(a, st); else bwd_t<TS, TexT, BGPP, false>(a, st);
}
template <int TS, typename TexT>
static void bwd_d1(const RasterArgs &a, hipStream_t st)
{
    if (a.bg_pp) bwd_d2<TS, TexT, true>(a, st); else bwd_d2<TS, TexT, false>(a, st);
}
template <int TS>
static void bwd_d0(const RasterArgs &a, hipStream_t st)
{
    if (a.dtype == 0) bwd_d1<TS, float>(a, st); else bwd_d1<TS, uint16_t>(a, st);
}

hipError_t launch_raster_fwd(const RasterArgs &a, hipStream_t st)
{
    if (a.n_tiles > 0) {
        switch (a.TS) {
        case 8: fwd_d0<8>(a, st); break;
        case 16: fwd_d0<16>(a, st); break;
        default: fwd_d0<32>(a, st); break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_raster_bwd(const RasterArgs &a, hipStream_t st)
{
    if (a.n_param_floats > 0)
        k_fill0<<<(unsigned)((a.n_param_floats + 255) / 256), 256, 0, st>>>(a.dparams,
                                                                             a.n_param_floats);
    if (a.n_tiles > 0) {
        switch (a.TS) {
        case 8: bwd_d0<8>(a, st); break;
        case 16: bwd_d0<16>(a, st); break;
        default: bwd_d0<32>(a, st); break;
        }
    }
    return hipGetLastError();
}

}  // namespace dbmp
