// Internal layouts and device helpers of the gfx950 rasteriser. Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dbmp {

// Device-side flag slots (int32 each) kept in the context workspace.
enum Flag : int {
    // per forward (reset at the start of every forward)
    F_OVERFLOW = 0,     // more (tile, primitive) pairs than the pair buffer holds
    F_BADIDX = 1,       // an atlas index outside [0, B)
    F_NONFINITE = 2,    // a non-finite parameter / texel / scale
    F_TOTAL = 3,        // number of (tile, primitive) pairs of this forward (clamped to INT_MAX)
    // sticky (raised by any forward; errors cleared by dbmp_check, the maximum by dbmp_reserve)
    F_S_OVERFLOW = 4,
    F_S_BADIDX = 5,
    F_S_NONFINITE = 6,
    F_S_TOTALMAX = 7,   // largest per-forward pair count since the last reserve
    F_COUNT = 16
};

// Transmittance threshold of the backward: layers in front of which T has fallen below TAU
// (2^-64) get a zero gradient; their exact gradient is below TAU times an O(1) factor.
#define DBMP_TAU 5.42101086242752217e-20f

// Per-tile pair counters are updated by device-scope atomics, which serialise per cache line;
// each counter therefore gets a 128-byte line of its own (tile t at tile_count[t * CNT_STRIDE]).
#define CNT_STRIDE 32

// The evaluated-pair counter is spread over this many 64-bit slots (summed when read).
#define DBMP_COUNTER_SLOTS 1024

// One image of a (possibly batched) launch.
struct ImgDev {
    int H, W, N;
    int ntx, nty;        // tiles along x and y
    int tile_off;        // first global tile index of this image
    int pad0, pad1;
    long long prim_off;  // first global primitive row
    long long pix_off;   // first global pixel (image planes at 3 * pix_off)
};

// Per-primitive record written by the setup kernel and read (wave-uniformly, through the scalar
// cache) by the raster kernels. Coordinates are those of the padded bitmap, where the texel
// (r, c) of Eq. (2) sits at padded (r + 1, c + 1):
//     U' = aU x + bU y + eU = U + 1,   V' = aV x + bV y + eV = V + 1.
struct __attribute__((aligned(16))) PrimRec {
    double aU, bU, eU;
    double aV, bV, eV;
    double Ulo, Uhi, Vlo, Vhi;  // M is non-zero only for Ulo <= U' < Uhi and Vlo <= V' < Vhi
    float ka;                   // alpha_max * sigmoid(nu)
    float cr, cg, cb;           // sigmoid of the colour logits
    int tex;                    // element offset of the padded bitmap's (0, 0)
    float omsig;                // 1 - sigmoid(nu)
    float faU, fbU, faV, fbV;   // float copies of the map's linear part (backward chain rule)
    int tx0, tx1, ty0, ty1;     // tile span of the support's bounding box (empty: tx0 > tx1)
    int img;
    int pad[3];
};
static_assert(sizeof(PrimRec) == 160, "PrimRec layout");

__device__ __forceinline__ int find_by_prim(const ImgDev *__restrict__ imgs, int n, long long g)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {  // last image whose prim_off <= g
        const int mid = (lo + hi + 1) >> 1;
        if (imgs[mid].prim_off <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int find_by_tile(const ImgDev *__restrict__ imgs, int n, int t)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (imgs[mid].tile_off <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Consecutive workgroup ids are dealt round-robin over the 8 XCDs; this bijection gives each
// XCD a contiguous run of tiles (a band of the image), so primitives shared by neighbouring
// tiles are fetched into the same L2.
__device__ __forceinline__ int xcd_remap(int bid, int n)
{
    const int q = n >> 3, r = n & 7;
    const int x = bid & 7, l = bid >> 3;
    return x * q + (x < r ? x : r) + l;
}

template <typename TexT> __device__ __forceinline__ float texel(TexT v);
template <> __device__ __forceinline__ float texel<float>(float v) { return v; }
template <> __device__ __forceinline__ float texel<uint16_t>(uint16_t v)
{
    return __uint_as_float(((uint32_t)v) << 16);  // bf16 -> f32 widening is exact
}

// Launch arguments shared by the host code and the launchers.
struct BinArgs {
    const float *params;
    const int *idx;
    long long n_rows;
    const ImgDev *imgs;
    int n_images;
    int n_tiles;
    const void *atlas;
    int dtype;  // 0 f32, 1 bf16
    int B, Hb, Wb, Wp;
    float alpha_max;
    int TS;
    void *atlas_pad;
    int *box;
    PrimRec *recs;
    int *tile_count, *tile_start;
    int *pairs;
    long long pair_cap;
    int *flags;
};

struct RasterArgs {
    const PrimRec *recs;
    const int *pairs, *tile_start, *tile_count;
    const ImgDev *imgs;
    int n_images, n_tiles;
    const void *atlas_pad;
    int dtype, Wp, Hb, Wb;
    const float *bg;
    int bg_pp;
    float *image, *alpha;
    int *saveK;
    float *saveT;
    const float *gI, *gA;
    float *dparams;
    long long n_param_floats;
    const int *flags;
    int TS;
    unsigned long long *pair_counter;  // cumulative count of evaluated (pixel, primitive) pairs
};

hipError_t launch_binning(const BinArgs &a, hipStream_t st);
hipError_t launch_raster_fwd(const RasterArgs &a, hipStream_t st);
hipError_t launch_raster_bwd(const RasterArgs &a, hipStream_t st);

}  // namespace dbmp
