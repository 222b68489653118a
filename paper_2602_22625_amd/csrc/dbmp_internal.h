// Internal layouts and device helpers of the gfx950 rasteriser. Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace dbmp {

// Device-side flag slots (int32 each) kept in the context workspace.
enum Flag : int {
    // Raised by any forward; cleared (and reported) by dbmp_check. A tile whose list did not
    // fit also knows it locally (its count exceeds the capacity) and renders nothing.
    F_S_OVERFLOW = 0,   // a tile's list is longer than the list capacity
    F_S_BADIDX = 1,     // an atlas index outside [0, B)
    F_S_NONFINITE = 2,  // a non-finite parameter / texel / scale
    F_COUNT = 16
};

// Transmittance threshold of the backward: layers in front of which T has fallen below TAU
// (2^-64) get a zero gradient; their exact gradient is below TAU times an O(1) factor.
#define DBMP_TAU 5.42101086242752217e-20f

// The evaluated-pair counter and the longest-list statistic are spread over this many slots
// (summed / max-reduced when read) so that no single address is hot.
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

// Per-primitive record written by the setup kernel and read by the raster kernels (staged in LDS
// per batch of list entries): only what the walks and the flush read, 160 bytes; the fields the
// forward needs come first. (The tile span and image fields of the binning stay in its LDS.) Coordinates are those
// of the padded bitmap, where the texel (r, c) of Eq. (2) sits at padded (r + 1, c + 1):
//     U' = aU x + bU y + eU = U + 1,   V' = aV x + bV y + eV = V + 1.
struct __attribute__((aligned(16))) PrimRec {
    double aU, bU, eU;
    double aV, bV, eV;
    double Ulo, Uhi, Vlo, Vhi;  // M is non-zero only for Ulo <= U' < Uhi and Vlo <= V' < Vhi
    int px0, px1, py0, py1;     // pixel bounding box of that region (empty: px0 > px1)
    float ka;                   // alpha_max * sigmoid(nu)
    float cr, cg, cb;           // sigmoid of the colour logits
    int tex;                    // element offset of the padded bitmap's (0, 0)
    float kaom;                 // alpha_max * sigmoid(nu) * (1 - sigmoid(nu))  (d alpha / d nu / M)
    float ccr, ccg, ccb;        // c (1 - c): derivative of the colour sigmoid
    float faU, fbU, faV, fbV;   // float copies of the map's linear part (backward chain rule)
    int id;                     // the primitive's row in params
    int pad[2];
};
static_assert(sizeof(PrimRec) == 160, "PrimRec layout");
static_assert(offsetof(PrimRec, px0) == 80, "the pixel box is read as one 16-byte vector");
static_assert(offsetof(PrimRec, ka) == 96 && offsetof(PrimRec, cb) == 108,
              "opacity and colour are read as one 16-byte vector");

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
template <> __device__ __forceinline__ float texel<_Float16>(_Float16 v) { return (float)v; }

// Launch arguments shared by the host code and the launchers.
// Adam applied by the binning to a gradient left pending by the previous fit step (see
// dbmp_fit_step): params non-null enables it.
struct AdamArgs {
    float *params, *grad, *m, *v;
    int *state;  // {updates applied, unused, gradient pending, unused}
    float lr, b1, b2, eps;
};

struct BinArgs {
    const float *params;
    const int *idx;
    long long n_rows;
    const ImgDev *imgs;
    int n_images;
    int n_tiles;
    const void *atlas;
    int dtype;  // 0 f32, 1 bf16, 2 f16 (the reduced-precision raster)
    int B, Hb, Wb, Wp;
    float alpha_max;
    int TS;
    void *atlas_pad;
    int *box;
    PrimRec *recs;
    int *tile_count;   // entries per tile list (zero on entry; the forward raster re-zeroes)
    int *lists;        // tile t's list at lists[t * list_cap]
    int list_cap;
    int *flags;
    bool pad_atlas;    // pad the atlas and find its boxes (false: reuse the stored ones)
    AdamArgs adam;     // adam.params non-null: apply the pending Adam update first
    int *order;        // non-null: tiles by decreasing list length are written here
    int *order_hist;   // ORDER_BINS x ceil(n_tiles / ORDER_CHUNK) ints (many-tile ordering)
    const int *prev_len;  // the previous forward's list lengths (any values: only the order uses them)
};

struct RasterArgs {
    const PrimRec *recs;
    const int *lists;
    int *tile_count;   // the forward reads each tile's count, stores it in tile_len, zeroes it
    int *tile_len;
    int list_cap;
    int *list_max;     // per-slot longest list seen since the last reserve
    const ImgDev *imgs;
    int n_images, n_tiles;
    const void *atlas_pad;
    int dtype, Wp, Hb, Wb;
    int zcell;                         // element offset of the padded atlas's all-zero cell
    int atlas_lds_bytes;               // > 0: the pipelined build stages this many bytes of the
                                       // padded atlas in LDS (dbmp_set_atlas_placement)
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
    const float *target;               // non-NULL: the backward forms the MSE gradient itself
    float *loss_tile;                  // per-tile sums of squared errors (MSE backward)
    int sched;                         // SCHED_GRID, SCHED_SORTED or SCHED_PERSISTENT
    int grid;                          // workgroups of a persistent launch
    int grab;                          // persistent: items per queue grab (0: static strides)
    const int *order;                  // tiles by decreasing list length (SORTED, PERSISTENT)
    int *queue;                        // persistent work queues: fwd {head, done}, bwd {head, done}
    hipEvent_t ev_start, ev_stop;      // non-null: recorded by the device around the raster launch
    int *fit_state;                    // fused fit step: its Adam state (counts the update the
                                       // binning applied; marks the new gradient pending)
    int n_cu;                          // compute units of the device (the walk form's choice)
};

// How the raster kernels map workgroups to tiles.
//   SCHED_GRID        one workgroup per tile, tiles in XCD-banded image order;
//   SCHED_SORTED      one workgroup per tile, tiles dealt longest list first;
//   SCHED_PERSISTENT  a fixed number of workgroups take tiles, longest list first, from a
//                     device queue until it is empty (or, with grab = 0, in fixed strides).
enum { SCHED_GRID = 0, SCHED_SORTED = 1, SCHED_PERSISTENT = 2 };

// workspace of the many-tile ordering (bin.hip): per-workgroup histograms of the list lengths
size_t order_hist_bytes(long long n_tiles);
hipError_t launch_binning(const BinArgs &a, hipStream_t st);
hipError_t launch_raster_fwd(const RasterArgs &a, hipStream_t st);
hipError_t launch_raster_bwd(const RasterArgs &a, hipStream_t st);
// the pipelined one-tile-per-workgroup build (raster_pipe.hip)
hipError_t launch_raster_fwd_pipe(const RasterArgs &a, hipStream_t st);
hipError_t launch_raster_bwd_pipe(const RasterArgs &a, hipStream_t st);
// the reduced-precision build (fp16 texels, packed fp16 bilinear blend), every launch form
// (raster_f16.hip); the backward's parameter gradient must already be cleared
hipError_t launch_raster_fwd_f16(const RasterArgs &a, hipStream_t st);
hipError_t launch_raster_bwd_f16(const RasterArgs &a, hipStream_t st);
hipError_t launch_fill0(float *p, long long n, hipStream_t st);
hipError_t launch_loss_sum(const float *loss_tile, const ImgDev *imgs, int n_images, float *out,
                           hipStream_t st);

}  // namespace dbmp
