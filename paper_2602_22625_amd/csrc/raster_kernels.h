// Forward and backward raster kernels (Sec. 3.1.1-3.1.2; Supp. Eqs. S1-S5).
//
// One workgroup per T x T screen tile, one lane per pixel, the tile's wave64s laid out as 8 x 8
// pixel blocks (the most compact footprint, so whole waves skip primitives they do not touch).
// The tile's list is walked in batches of 64 entries whose records the workgroup first copies to
// LDS; each wave then visits only the entries whose pixel box overlaps its block. Texels are fetched
// from the zero-bordered atlas copy (L1/L2): at these workloads a primitive is minified 2-8x,
// so staging its footprint in LDS would move many more texels than the 4 each pixel samples.
//
// Precision: the canvas -> bitmap map is evaluated in float64 (2 FMAs per coordinate; on
// gfx950 a float64 FMA issues at the rate of a non-packed float32 one), so the bilinear weights
// carry float32 precision even at U ~ 128; sampling and compositing are float32. Inside the
// support U', V' >= 0, so the texel index is the truncation and the weight the fraction.
//
// Forward: the workgroup first sorts its tile's list ascending (front to back) in LDS and
// writes it back for the backward, then composites C += T alpha c, T *= (1 - alpha) (Eqs. 4-5),
// I = C + T b, A = 1 - T. It stores no per-layer state; per pixel it keeps the list position K
// of the last layer in front of which T >= TAU, and T_K.
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
// The 8 per-lane factors are reduced across the wave by a transposed butterfly built from
// gfx950's cross-row lane swaps (v_permlane32_swap, v_permlane16_swap) and DPP row/quad
// permutes, after which lane 8q holds the wave total of factor q; eight lanes add them into the
// workgroup's per-entry LDS sums, which after each batch are scaled by the primitive's constant
// factors and flushed with one float32 atomic per (tile entry, parameter). Since g is fixed per
// pixel, the walk carries only the scalar g . G of the composite behind each layer.
//
// Each walk comes in two builds (LAUNCH below): one texel cell in flight, or two, where the
// next visited entry's texels are requested before the current entry is processed.
#pragma once

#include "dbmp_internal.h"

#include <hip/hip_ext.h>

#include <limits.h>

#include <algorithm>
#include <type_traits>

// x * y, except that 0 times anything (infinity and NaN included) is 0 (v_mul_legacy_f32). The
// compiler's own intrinsic, not inline assembly, so that it sees the instruction: on gfx950 a
// vector instruction that reads a reciprocal's result in the next cycle needs a wait state,
// which the compiler inserts only for instructions it knows.
extern "C" __device__ __attribute__((const)) float dbmp_mul_legacy(float, float) __asm(
    "llvm.amdgcn.fmul.legacy");

namespace dbmp {

template <int TS>
struct TileGeom {
    int px, py, pix;
    bool valid;
    ImgDev D;
    int b;
    int bx0, by0;  // origin of this wave's 8 x 8 pixel block (wave-uniform)
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
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    tg.bx0 = tx * TS + (wave % WPR) * 8;
    tg.by0 = ty * TS + (wave / WPR) * 8;
    tg.px = tg.bx0 + (lane & 7);
    tg.py = tg.by0 + (lane >> 3);
    tg.valid = tg.px < tg.D.W && tg.py < tg.D.H;
    tg.pix = tg.py * tg.D.W + tg.px;
    return tg;
}

// List entries are processed in batches of 64: the workgroup copies the batch's records into LDS
// with coalesced 16-byte loads (independent, so their latencies overlap), then every wave marks
// with one ballot the entries whose pixel box overlaps its 8 x 8 block (lane e tests entry e)
// and visits only those, reading the record from LDS.
constexpr int BATCH = 64;
constexpr int RQ = sizeof(PrimRec) / 16;

template <int NT, typename IdAt>
__device__ __forceinline__ void stage_batch(PrimRec *__restrict__ s_rec,
                                            const PrimRec *__restrict__ recs, int b0, int cnt,
                                            IdAt id_at)
{
    const uint4 *src = reinterpret_cast<const uint4 *>(recs);
    uint4 *dst = reinterpret_cast<uint4 *>(s_rec);
    for (int q = threadIdx.x; q < cnt * RQ; q += NT) {
        const int e = q / RQ;
        dst[q] = src[(size_t)id_at(b0 + e) * RQ + (q - e * RQ)];
    }
}

__device__ __forceinline__ uint64_t batch_hits(const PrimRec *__restrict__ s_rec, int cnt, int bx0,
                                               int by0)
{
    const int e = threadIdx.x & 63;
    bool hit = false;
    if (e < cnt) {
        const int4 bb = *reinterpret_cast<const int4 *>(&s_rec[e].px0);  // px0, px1, py0, py1
        hit = bb.y >= bx0 && bb.x <= bx0 + 7 && bb.w >= by0 && bb.z <= by0 + 7;
    }
    return __ballot(hit);
}

// Lanes of the wave whose pixel lies in the primitive's support: four float64 compares whose
// lane masks are combined on the scalar unit.
__device__ __forceinline__ uint64_t support_mask(const PrimRec &r, double U, double V,
                                                 uint64_t valid)
{
    return __ballot(U >= r.Ulo) & __ballot(U < r.Uhi) & __ballot(V >= r.Vlo) &
           __ballot(V < r.Vhi) & valid;
}

// Bilinear sampling of the padded bitmap at (U', V') >= 0 (Supp. Eqs. S1-S3), in two steps so
// that a walk can request the next entry's cell before it blends the current one: request_cell
// issues the four texel loads (kept as stored: converting them here would wait for them), blend
// forms M and its derivatives along U' and V'. Forward and backward evaluate the same arithmetic,
// so both obtain bit-identical alpha (the backward's transmittance recovery relies on it).
template <typename TexT>
struct Cell {
    TexT p00, p01, p10, p11;  // texels (iu, iv), (iu + 1, iv), (iu, iv + 1), (iu + 1, iv + 1)
    float wu, wv;             // fractional position inside the cell
};

// The reduced-precision build (fp16 texels, Sec. 3.1.2's half-precision path): the two texels of
// a cell row are adjacent, so each row is one 4-byte load (gfx950 serves unaligned dword loads),
// and the pair stays packed for the blend. The weights are packed too, rounded toward zero.
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
template <>
struct Cell<_Float16> {
    half2v A, B;  // (p00, p01) and (p10, p11)
    half2v w;     // (wu, wv)
};
template <typename TexT>
constexpr bool is_f16 = std::is_same<TexT, _Float16>::value;

// A lane outside the support (in = false) reads the all-zero cell that follows the padded
// atlas (element offset zcell), so M = MU = MV = 0 there exactly whatever its weights: one
// select of the address, no select of the weights. The cell is addressed by its 32-bit byte
// offset from the atlas base (atlases are below 4 GB): the loads take the base from scalar
// registers and only the offset per lane, and the offset costs one 24-bit multiply-add (texel
// coordinates and row pitches are below 2^24). Inside the support U', V' >= 0: the texel index
// is the truncation.
// PIN (pipelined walks): the loads stay where they are issued, ahead of the other cell's
// arithmetic, instead of being moved down to their first use by the compiler.
// LDSA: `atlas` points to the workgroup's LDS copy of the padded atlas (LDS reads).
template <typename TexT, bool PIN, bool LDSA = false>
__device__ __forceinline__ void request_cell(Cell<TexT> &c, const TexT *__restrict__ atlas,
                                             int tex, int Wp, double U, double V, bool in,
                                             int zcell)
{
    const float wu = (float)__builtin_amdgcn_fract(U), wv = (float)__builtin_amdgcn_fract(V);
    if constexpr (is_f16<TexT>)
        c.w = __builtin_bit_cast(half2v, __builtin_amdgcn_cvt_pkrtz(wu, wv));
    else {
        c.wu = wu;
        c.wv = wv;
    }
    const unsigned at = in ? (unsigned)tex + __umul24((unsigned)(int)V, (unsigned)Wp) +
                                 (unsigned)(int)U
                           : (unsigned)zcell;
    const unsigned b0 = at * (unsigned)sizeof(TexT);
    // the row below as a 64-bit offset: the compiler adds the pitch to the scalar base, and
    // both loads take the same per-lane offset b0
    const size_t b1 = (size_t)b0 + (size_t)Wp * sizeof(TexT);
    auto load = [&](auto *t0, auto *t1) {
        if constexpr (is_f16<TexT>) {  // merged by the compiler into one dword load per row
            c.A = half2v{t0[0], t0[1]};
            c.B = half2v{t1[0], t1[1]};
        } else {
            c.p00 = t0[0];
            c.p01 = t0[1];
            c.p10 = t1[0];
            c.p11 = t1[1];
        }
    };
    // The atlas is a read-only kernel argument, so the compiler takes loads from it as
    // movable anywhere; seen through this (empty) statement the base is an ordinary pointer,
    // and the loads stay ahead of the statement at the end.
    if constexpr (LDSA) {
        using LChar = const __attribute__((address_space(3))) char;
        using LTex = const __attribute__((address_space(3))) TexT;
        LChar *base = (LChar *)atlas;
        if constexpr (PIN) asm volatile("" : "+s"(base));
        load((LTex *)(base + b0), (LTex *)(base + b1));
    } else {
        using GChar = const __attribute__((address_space(1))) char;
        using GTex = const __attribute__((address_space(1))) TexT;
        GChar *base = (GChar *)atlas;
        if constexpr (PIN) asm volatile("" : "+s"(base));
        load((GTex *)(base + b0), (GTex *)(base + b1));
    }
    // no instruction and no wait: only an ordering point for the compiler
    if constexpr (PIN) asm volatile("" ::: "memory");
}

// Waits for a requested cell that will not be blended (the last request of a batch), so that
// no load into its registers is still outstanding when the next batch reuses them.
template <typename TexT>
__device__ __forceinline__ void drop_cell(const Cell<TexT> &c)
{
    if constexpr (is_f16<TexT>)
        asm volatile("" ::"v"(c.A), "v"(c.B));
    else
        asm volatile("" ::"v"(c.p00), "v"(c.p01), "v"(c.p10), "v"(c.p11));
}

// The bilinear value M and its derivatives M_U, M_V of one sample: float32, or (fp16 build) the
// two packed registers the blend leaves, W = (M, M_V) and Z = (M_U, unused), widened on use.
template <typename TexT>
struct Bil {
    float M, MU, MV;
    __device__ float m() const { return M; }
    __device__ float mu() const { return MU; }
    __device__ float mv() const { return MV; }
};
template <>
struct Bil<_Float16> {
    half2v W, Z;
    __device__ float m() const { return (float)W.x; }
    __device__ float mu() const { return (float)Z.x; }
    __device__ float mv() const { return (float)W.y; }
};

template <typename TexT>
__device__ __forceinline__ Bil<TexT> blend(const Cell<TexT> &c)
{
    Bil<TexT> b;
    if constexpr (is_f16<TexT>) {
        // packed fp16 (v_pk_fma_f16): interpolate both columns along V' first, then along U'
        const half2v wu = {c.w.x, c.w.x}, wv = {c.w.y, c.w.y};
        const half2v E = c.B - c.A;                             // (p10 - p00, p11 - p01)
        const half2v R = __builtin_elementwise_fma(wv, E, c.A);  // the column values at V'
        const half2v X = __builtin_shufflevector(R, E, 0, 2);
        const half2v Y = __builtin_shufflevector(R, E, 1, 3);
        b.Z = Y - X;                                             // (M_U, e1 - e0)
        b.W = __builtin_elementwise_fma(wu, b.Z, X);             // (M, M_V)
    } else {
        const float p00 = texel<TexT>(c.p00), p01 = texel<TexT>(c.p01);
        const float p10 = texel<TexT>(c.p10), p11 = texel<TexT>(c.p11);
        const float d0 = p01 - p00, d1 = p11 - p10;
        const float top = fmaf(c.wu, d0, p00);
        const float bot = fmaf(c.wu, d1, p10);
        b.MV = bot - top;
        b.M = fmaf(c.wv, b.MV, top);
        b.MU = fmaf(c.wv, d1 - d0, d0);
    }
    return b;
}

// Visits per wave whose bilinear values the fused step keeps for its backward (3 vector
// registers each; 0 keeps none). Six keep the fused 16 x 16 kernel at 72 vector registers,
// 7 waves per SIMD; at 2048^2 it took 175 us against 193 us with none and 184 us with four,
// while eight (84 registers, 5 waves) took 196 us.
#ifndef STORED_VISITS
#define STORED_VISITS 6
#endif
// The same for the pipelined build, which runs where the grid itself holds at most 4 waves per
// SIMD, so registers are not the limit there up to 128 (even number: the walk stores visits in
// pairs). Ten keep the 16 x 16 build at 90 vector registers with no scalar-register spill
// (twelve spill scalar registers).
#ifndef STORED_VISITS_PIPE
#define STORED_VISITS_PIPE 10
#endif
// The fp16 build keeps a visit in 2 vector registers instead of 3 (its entry index takes a
// scalar register either way): 7 keep the fused 16 x 16 kernel at 72 vector registers, 7 waves
// per SIMD, and the pipelined build stays without scalar spills up to 10 (80 registers).
#ifndef STORED_VISITS_F16
#define STORED_VISITS_F16 7
#endif
#ifndef STORED_VISITS_PIPE_F16
#define STORED_VISITS_PIPE_F16 10
#endif

// Lists up to this length are sorted in LDS, longer ones in place in global memory. At 512
// entries for 8 x 8 and 16 x 16 tiles the buffer takes 2 KB; at 2,048 it limited the 16 x 16
// forward to 7 workgroups per CU by LDS (lists at these workloads are far shorter).
template <int TS>
struct SortCap {
    static constexpr int v = TS == 32 ? 4096 : 512;
};

// Ascending bitonic network with only ascending comparators (the first sub-stage of every merge
// compares i with i ^ (k - 1)): a list of any length n behaves as if padded with +inf, and
// comparators reaching past n are skipped. Executed by all NT threads of the workgroup.
template <int NT, typename Get, typename Set, typename Sync>
__device__ __forceinline__ void bitonic_sort(int n, Get get, Set set, Sync sync)
{
    int N2 = 1;
    while (N2 < n) N2 <<= 1;
    for (int k = 2; k <= N2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < N2; i += NT) {
                const int l = (j == (k >> 1)) ? (i ^ (k - 1)) : (i ^ j);
                if (l > i && l < n) {
                    const int x = get(i), y = get(l);
                    if (y < x) { set(i, y); set(l, x); }
                }
            }
            sync();
        }
    }
}

// ------------------------------------------------------------------------------------------
// Wave reduction of 8 values per lane.
// ------------------------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}

// Transposed butterfly: v_permlane32_swap leaves values 0-3 summed over lanes l and l^32 in the
// low half and values 4-7 in the high half; v_permlane16_swap halves again across rows; a
// row_mirror step (with a select) across the two 8-lane halves of a row; then row_half_mirror,
// quad_perm [1,0,3,2] and [2,3,0,1] add within groups of 8. On return lane l holds the wave
// total of value (l >> 3). 18 VALU instructions, no LDS.
__device__ __forceinline__ float reduce8(const float (&v)[8], int lane)
{
    float w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]),
                                                        __float_as_uint(v[i + 4]), false, false);
        w[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    float x[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(w[i]),
                                                        __float_as_uint(w[i + 2]), false, false);
        x[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    const bool h3 = lane & 8;
    float y = (h3 ? x[1] : x[0]) + dpp<0x140>(h3 ? x[0] : x[1]);  // row_mirror
    y += dpp<0x141>(y);                                            // row_half_mirror
    y += dpp<0xB1>(y);                                             // quad_perm [1,0,3,2]
    y += dpp<0x4E>(y);                                             // quad_perm [2,3,0,1]
    return y;
}

// Sum of one value over the wave (result valid in every lane).
__device__ __forceinline__ float wave_sum(float y)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(y), __float_as_uint(y), false,
                                                    false);
    y = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    const auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(y), __float_as_uint(y), false,
                                                    false);
    y = __uint_as_float(q[0]) + __uint_as_float(q[1]);
    y += dpp<0x140>(y);
    y += dpp<0x141>(y);
    y += dpp<0xB1>(y);
    y += dpp<0x4E>(y);
    return y;
}

// Runs `body(tile)` for the tiles this workgroup owns under the launch schedule (see SCHED_*).
// Persistent with grab > 0: thread 0 takes the next `grab` items from the queue and shares the
// first through LDS; the barrier at the top of each round also guarantees every lane has
// finished the previous tile before its LDS is reused. The last workgroup to leave re-arms the
// queue for the next launch. Persistent with grab == 0: workgroup w takes items w, w + G,
// w + 2G, ... of the longest-first order (no atomics; the order balances the strides).
// PERSIST is a compile-time choice: a kernel built for the one-tile-per-workgroup schedules
// carries none of the persistent loop's state, which keeps it at about 60 scalar registers
// instead of over 100 (a limit on waves per SIMD).
// How a raster kernel is built (a template argument, chosen per launch by the host):
//   LAUNCH_TILE        one tile per workgroup (grid and sorted schedules), one cell in flight;
//   LAUNCH_PERSISTENT  the persistent schedule's loop;
//   LAUNCH_TILE_PIPE   one tile per workgroup, and the walks keep a second cell in flight: the
//                      next visited entry's texels are requested before the current entry is
//                      processed. This hides the texel latency where few waves share a SIMD
//                      (small canvases); where the SIMDs are full of waves, they hide it, and
//                      the second cell's instructions and registers only cost.
//   LAUNCH_TILE_PIPE_LDS  the pipelined build reading its texels from a copy of the padded atlas
//                      that every workgroup stages in LDS first (small atlases, on request:
//                      dbmp_set_atlas_placement).
enum { LAUNCH_TILE = 0, LAUNCH_PERSISTENT = 1, LAUNCH_TILE_PIPE = 2, LAUNCH_TILE_PIPE_LDS = 3 };

// The LDS copy of the padded atlas (LAUNCH_TILE_PIPE_LDS): `bytes` of it, copied by the whole
// workgroup with 4-byte loads (element sizes are 2 or 4 bytes; an odd trailing 2-byte element
// is copied alone), then a barrier. Returns the copy's base.
template <typename TexT>
__device__ __forceinline__ const TexT *stage_atlas(const TexT *__restrict__ atlas, int bytes)
{
    extern __shared__ __attribute__((aligned(16))) uint32_t s_atlas[];
    const uint32_t *src = reinterpret_cast<const uint32_t *>(atlas);
    const int words = bytes >> 2;
    for (int i = threadIdx.x; i < words; i += blockDim.x) s_atlas[i] = src[i];
    if ((bytes & 3) && threadIdx.x == 0)
        reinterpret_cast<uint16_t *>(s_atlas)[2 * words] =
            reinterpret_cast<const uint16_t *>(atlas)[2 * words];
    __syncthreads();
    return reinterpret_cast<const TexT *>(s_atlas);
}

template <bool PERSIST, typename Body>
__device__ __forceinline__ void run_schedule(int sched, int grab, const int *__restrict__ order,
                                             int *__restrict__ queue, int n_tiles, Body body)
{
    if constexpr (!PERSIST) {
        body(sched == SCHED_SORTED ? order[blockIdx.x] : xcd_remap(blockIdx.x, n_tiles));
        return;
    }
    if (grab == 0) {
        for (int item = blockIdx.x; item < n_tiles; item += gridDim.x) {
            __syncthreads();  // the previous tile's LDS is free
            body(order[item]);
        }
        return;
    }
    __shared__ int s_item;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(queue, grab);
        __syncthreads();
        const int first = s_item;
        if (first >= n_tiles) break;  // every workgroup reaches this once the queue is drained
        const int last = min(first + grab, n_tiles);
        for (int item = first; item < last; ++item) {
            if (item > first) __syncthreads();
            body(order[item]);
        }
    }
    // No fence: no data flows through the queue, and the last workgroup to leave knows that
    // every other one has taken its final item (it left the loop before counting itself out).
    if (threadIdx.x == 0 &&
        __hip_atomic_fetch_add(queue + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
            (int)gridDim.x - 1) {
        queue[0] = 0;
        queue[1] = 0;
    }
}

// Visits whose per-lane bilinear values (M and its derivatives along U' and V') the fused
// step's forward keeps in registers for its own backward: the first SV visits of a list that
// fits one batch. The backward then neither repeats the support test nor fetches and blends the
// texels of those visits; it only recomputes U', V' for the geometric terms. Lanes outside a
// visit's support sampled the all-zero cell, so their stored values are exactly 0. SV = 1 with
// n = 0 is the form that stores nothing.
template <int SV, typename TexT>
struct Stored {
    Bil<TexT> b[SV];
    int e[SV];
    int n = 0;     // visits stored
    int last = -1; // the last stored visit's batch entry (visits go in ascending entry order)
};

// FUSED: the forward of a fit step, followed in the same workgroup by the backward of the MSE
// loss against `target` (the image, the per-pixel (K, T_K) and, for a list of at most 64
// entries, the staged records are still on chip); the gradient is added to dparams and the
// tile's squared error written to loss_tile.
// The backward's walk over a tile's sorted list (defined below, after the forward kernel that
// also runs it in the fused fit step).
template <int NT, typename TexT, bool HAS_GA, bool PIPE, bool LDSA, int TS, int SV,
          typename IdAt>
__device__ __forceinline__ void bwd_walk(int n, IdAt id_at, bool staged,
                                         const Stored<SV, TexT> &st,
                                         PrimRec *__restrict__ s_rec,
                                         float *__restrict__ s_grad,
                                         const PrimRec *__restrict__ recs,
                                         const TexT *__restrict__ atlas, int Wp, int zcell,
                                         const TileGeom<TS> &tg, uint64_t vmask, float g0,
                                         float g1, float g2, float ga, float G0, float G1,
                                         float G2, int K, float TK, float *__restrict__ dparams,
                                         double cu1, double cv1, float cu_cv2, float cv_cu,
                                         int lane);

template <int TS, typename TexT, bool BG_PP, bool FUSED, int LAUNCH>
__global__ void __launch_bounds__(TS * TS)
k_raster_fwd(const PrimRec *__restrict__ recs, int *__restrict__ lists, int list_cap,
             int *__restrict__ tile_count, int *__restrict__ tile_len, int *__restrict__ list_max,
             const ImgDev *__restrict__ imgs, int n_images, int n_tiles,
             const TexT *__restrict__ atlas_g, int Wp, int zcell, const float *__restrict__ bg,
             float *__restrict__ image, float *__restrict__ alpha, int *__restrict__ saveK,
             float *__restrict__ saveT, const int *__restrict__ flags,
             unsigned long long *__restrict__ pair_counter, int sched, int grab,
             const int *__restrict__ order, int *__restrict__ queue,
             const float *__restrict__ target, float *__restrict__ loss_tile,
             float *__restrict__ dparams, double cu1, double cv1, float cu_cv2, float cv_cu,
             int *__restrict__ fit_state, int atl_bytes)
{
    constexpr int NT = TS * TS, CAP = SortCap<TS>::v;
    constexpr bool LDSA = LAUNCH == LAUNCH_TILE_PIPE_LDS;
    constexpr bool PERSIST = LAUNCH == LAUNCH_PERSISTENT;
    constexpr bool PIPE = LAUNCH == LAUNCH_TILE_PIPE || LDSA;
    // the fused step keeps its first visits' bilinear values for the backward (the pipelined
    // build runs where the grid leaves SIMDs with few waves, so registers are not its limit)
    constexpr int SVN = (LAUNCH == LAUNCH_TILE || LAUNCH == LAUNCH_PERSISTENT)
                            ? (is_f16<TexT> ? STORED_VISITS_F16 : STORED_VISITS)
                        : PIPE ? (is_f16<TexT> ? STORED_VISITS_PIPE_F16 : STORED_VISITS_PIPE)
                               : 0;
    constexpr bool STORE = FUSED && SVN > 0;
    constexpr int SV = STORE ? SVN : 1;
    // A fit step's Adam state {updates applied, unused, gradient pending, unused}: this step's
    // binning applied the pending update if one was marked (count it), and this launch leaves a
    // new gradient pending. One thread, after the binning has ended (stream order) and before
    // the next step's binning reads the state.
    if (FUSED && fit_state && blockIdx.x == 0 && threadIdx.x == 0) {
        if (fit_state[2]) fit_state[0] += 1;
        fit_state[2] = 1;
    }
    __shared__ __attribute__((aligned(16))) int s_ids[CAP + 4];
    __shared__ PrimRec s_rec[BATCH];
    __shared__ float s_loss[TS * TS / 64];
    __shared__ float s_grad[FUSED ? BATCH * 8 : 1];  // the backward's per-entry partial sums
    if constexpr (FUSED) {
        for (int i = threadIdx.x; i < BATCH * 8; i += NT) s_grad[i] = 0.f;
        __syncthreads();
    }
    const TexT *atlas = atlas_g;
    if constexpr (LDSA) atlas = stage_atlas<TexT>(atlas_g, atl_bytes);
    auto tile_body = [&](const int tile) {
        const int n = tile_count[tile];
        __syncthreads();  // every lane has read the count before it is re-armed
        if (threadIdx.x == 0) {
            tile_count[tile] = 0;  // ready for the next forward's appends
            tile_len[tile] = n;    // for the backward
            atomicMax(list_max + (blockIdx.x & (DBMP_COUNTER_SLOTS - 1)), n);  // statistic
        }
        if (n > list_cap) return;  // this tile's list did not fit (reported by dbmp_check)
        const TileGeom<TS> tg = tile_geom<TS>(tile, imgs, n_images);
        // the fused step's target pixel, requested now so that its latency passes during the
        // walks (it is used after the forward, to form dL/dI)
        float tq0 = 0.f, tq1 = 0.f, tq2 = 0.f;
        if (FUSED && tg.valid) {
            using GFloat = const __attribute__((address_space(1))) float;
            GFloat *tgt = (GFloat *)target;
            asm volatile("" : "+s"(tgt));  // an ordinary pointer: the loads stay here
            const size_t tplane = (size_t)tg.D.H * tg.D.W;
            GFloat *tp = tgt + 3 * tg.D.pix_off + tg.pix;
            tq0 = tp[0];
            tq1 = tp[tplane];
            tq2 = tp[2 * tplane];
            asm volatile("" ::: "memory");
        }
        int *seg = lists + (size_t)tile * list_cap;
        const bool in_lds = n <= CAP;

        // ---- sort the tile's list front to back (index order) and write it back -----------------
        if (in_lds) {
            for (int i = threadIdx.x; i < n + 4; i += NT) s_ids[i] = i < n ? seg[i] : INT_MAX;
            __syncthreads();
            if (n <= NT) {  // rank sort: entries are distinct primitive ids
                int v = INT_MAX, rank = 0;
                if ((int)threadIdx.x < n) {
                    v = s_ids[threadIdx.x];
                    for (int k = 0; k < n; k += 4) {
                        const int4 q = *reinterpret_cast<const int4 *>(&s_ids[k]);
                        rank += (q.x < v) + (q.y < v) + (q.z < v) + (q.w < v);
                    }
                }
                __syncthreads();
                if ((int)threadIdx.x < n) s_ids[rank] = v;
            } else {
                bitonic_sort<NT>(n, [&](int i) { return s_ids[i]; },
                                 [&](int i, int x) { s_ids[i] = x; }, [] { __syncthreads(); });
            }
            __syncthreads();
            for (int i = threadIdx.x; i < n; i += NT) seg[i] = s_ids[i];
        } else {  // longer than the LDS buffer: sort in place in global memory
            volatile int *vs = seg;
            bitonic_sort<NT>(n, [&](int i) { return vs[i]; }, [&](int i, int x) { vs[i] = x; },
                             [] { __threadfence_block(); __syncthreads(); });
        }

        // ---- composite ------------------------------------------------------------------------
        const double xd = tg.px, yd = tg.py;
        const uint64_t vmask = __ballot(tg.valid);
        float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, TK = 1.f;
        int K = -1;
        unsigned long long npairs = 0;  // wave-uniform count of evaluated (pixel, primitive) pairs
        // The next staged entry (ascending list order: front to back) that a lane of this wave
        // lies in, or -1, with the lanes in its support (m) and their bitmap coordinates.
        auto find = [&](uint64_t &hits, double &U, double &V, uint64_t &m) {
            m = 0;
            while (hits) {
                const int k = __builtin_ctzll(hits);
                hits &= hits - 1;
                const PrimRec &r = s_rec[k];
                U = fma(r.aU, xd, fma(r.bU, yd, r.eU));
                V = fma(r.aV, xd, fma(r.bV, yd, r.eV));
                m = support_mask(r, U, V, vmask);
                if (m != 0) {  // else no lane of this wave touches the primitive
                    npairs += __popcll(m);
                    return k;
                }
            }
            return -1;
        };
        // The pipelined walk requests a cell for every lane (and for the failed search that
        // ends a batch: entry -1, any valid bitmap, all weights zero), so that each cell's loads
        // are issued on every path ahead of the other cell's compositing.
        auto find_req = [&](uint64_t &hits, Cell<TexT> &c, uint64_t &m) {
            double U = 0.0, V = 0.0;
            const int e = find(hits, U, V, m);
            request_cell<TexT, true, LDSA>(c, atlas, e >= 0 ? s_rec[e].tex : 0, Wp, U, V,
                                           __builtin_amdgcn_inverse_ballot_w64(m), zcell);
            return e;
        };
        // The pipelined walk composites on every lane (no branch, so the wait for a cell's
        // texels is the same on every path): outside the support alpha = 0, which leaves C and
        // T exactly as they were; only the record of K is confined to the support. The other
        // walk evaluates the same arithmetic on the support lanes only.
        auto over_m = [&](int j, const PrimRec &r, float M, uint64_t m) {
            const float a = r.ka * M;  // Eq. (3)
            if (__builtin_amdgcn_inverse_ballot_w64(m) && T >= DBMP_TAU) { K = j; TK = T; }
            const float w = T * a;
            C0 = fmaf(w, r.cr, C0);
            C1 = fmaf(w, r.cg, C1);
            C2 = fmaf(w, r.cb, C2);
            T = fmaf(-T, a, T);  // T (1 - alpha), rounded once
        };
        auto over = [&](int j, const PrimRec &r, const Cell<TexT> &c, uint64_t m) {
            over_m(j, r, blend<TexT>(c).m(), m);
        };
        Stored<SV, TexT> st;
        auto composite = [&](auto id_at) {
            for (int b0 = 0; b0 < n; b0 += BATCH) {
                const int cnt = min(BATCH, n - b0);
                __syncthreads();  // the previous batch is consumed (first pass: the sort is done)
                stage_batch<NT>(s_rec, recs, b0, cnt, id_at);
                __syncthreads();
                uint64_t hits = batch_hits(s_rec, cnt, tg.bx0, tg.by0);
                if constexpr (PIPE) {
                    // two cells in turn: the next entry's texels are in flight while the
                    // current one is composited (the last request of a batch is dropped)
                    Cell<TexT> ca, cb;
                    uint64_t ma, mb;
                    int ea = find_req(hits, ca, ma);
                    if constexpr (STORE) {
                        // a list of one batch: its first SV visits (the same pipelined walk,
                        // unrolled two at a time) keep M, M_U, M_V for the backward
                        static_assert(SV % 2 == 0, "stored visits go in pairs");
                        if (n <= BATCH) {
#pragma unroll
                            for (int v = 0; v < SV; v += 2) {
                                if (ea < 0) break;
                                const int eb = find_req(hits, cb, mb);
                                {
                                    const Bil<TexT> b = blend<TexT>(ca);
                                    over_m(b0 + ea, s_rec[ea], b.m(), ma);
                                    st.b[v] = b;
                                    st.e[v] = ea; st.n = v + 1; st.last = ea;
                                }
                                if (eb < 0) { drop_cell(cb); ea = -1; break; }
                                ea = find_req(hits, ca, ma);
                                {
                                    const Bil<TexT> b = blend<TexT>(cb);
                                    over_m(b0 + eb, s_rec[eb], b.m(), mb);
                                    st.b[v + 1] = b;
                                    st.e[v + 1] = eb; st.n = v + 2; st.last = eb;
                                }
                            }
                        }
                    }
                    while (ea >= 0) {
                        const int eb = find_req(hits, cb, mb);
                        over(b0 + ea, s_rec[ea], ca, ma);
                        if (eb < 0) { drop_cell(cb); break; }
                        ea = find_req(hits, ca, ma);
                        over(b0 + eb, s_rec[eb], cb, mb);
                    }
                } else {
                    if constexpr (STORE) {
                        // a list of one batch: its first visits composite on every lane (the
                        // all-zero cell outside the support) and keep M, M_U, M_V for the
                        // backward of this workgroup
                        if (n <= BATCH) {
#pragma unroll
                            for (int v = 0; v < SV; ++v) {
                                double U, V;
                                uint64_t m;
                                const int e = find(hits, U, V, m);
                                if (e < 0) break;
                                const PrimRec &r = s_rec[e];
                                Cell<TexT> c;
                                request_cell<TexT, false, LDSA>(c, atlas, r.tex, Wp, U, V,
                                                          __builtin_amdgcn_inverse_ballot_w64(m),
                                                          zcell);
                                const Bil<TexT> b = blend<TexT>(c);
                                over_m(b0 + e, r, b.m(), m);
                                st.b[v] = b;
                                st.e[v] = e;
                                st.n = v + 1;
                                st.last = e;
                            }
                        }
                    }
                    while (hits) {  // ascending list order: front to back
                        const int e = __builtin_ctzll(hits);
                        hits &= hits - 1;
                        const PrimRec &r = s_rec[e];
                        const double U = fma(r.aU, xd, fma(r.bU, yd, r.eU));
                        const double V = fma(r.aV, xd, fma(r.bV, yd, r.eV));
                        const uint64_t m = support_mask(r, U, V, vmask);
                        if (m == 0) continue;  // no lane of this wave touches the primitive
                        npairs += __popcll(m);
                        if (__builtin_amdgcn_inverse_ballot_w64(m)) {  // the support lanes only
                            Cell<TexT> c;
                            request_cell<TexT, false, LDSA>(c, atlas, r.tex, Wp, U, V, true,
                                                            zcell);
                            const float a = r.ka * blend<TexT>(c).m();  // Eq. (3)
                            if (T >= DBMP_TAU) { K = b0 + e; TK = T; }
                            const float w = T * a;
                            C0 = fmaf(w, r.cr, C0);
                            C1 = fmaf(w, r.cg, C1);
                            C2 = fmaf(w, r.cb, C2);
                            T = fmaf(-T, a, T);
                        }
                    }
                }
            }
    };
    if (in_lds)
        composite([&](int j) { return s_ids[j]; });
    else
        composite([&](int j) { return ((volatile int *)seg)[j]; });
    if ((threadIdx.x & 63) == 0 && npairs)  // spread over slots: no single hot address
        atomicAdd(pair_counter + ((blockIdx.x * (NT / 64) + (threadIdx.x >> 6)) &
                                  (DBMP_COUNTER_SLOTS - 1)),
                  npairs);
    const ImgDev &D = tg.D;
    const size_t plane = (size_t)D.H * D.W;
    float b0 = 0.f, b1 = 0.f, b2 = 0.f;
    if (tg.valid) {
        if (BG_PP) {
            const float *bp = bg + 3 * D.pix_off + tg.pix;
            b0 = bp[0]; b1 = bp[plane]; b2 = bp[2 * plane];
        } else {
            b0 = bg[3 * tg.b]; b1 = bg[3 * tg.b + 1]; b2 = bg[3 * tg.b + 2];
        }
    }
    const float I0 = fmaf(T, b0, C0), I1 = fmaf(T, b1, C1), I2 = fmaf(T, b2, C2);
    const long long gp = D.pix_off + tg.pix;
    if (tg.valid) {
        float *ip = image + 3 * D.pix_off + tg.pix;
        ip[0] = I0;
        ip[plane] = I1;
        ip[2 * plane] = I2;
        if (alpha) alpha[gp] = 1.f - T;
        saveK[gp] = K;
        saveT[gp] = TK;
    }
    if constexpr (FUSED) {
        // dL/dI of the image's MSE, formed as the separate MSE backward forms it
        float g0 = 0.f, g1 = 0.f, g2 = 0.f, sq = 0.f;
        if (tg.valid) {
            const float e0 = I0 - tq0, e1 = I1 - tq1, e2 = I2 - tq2;
            sq = fmaf(e0, e0, fmaf(e1, e1, e2 * e2));
            const float sc = 2.f / (3.f * (float)plane);
            g0 = sc * e0; g1 = sc * e1; g2 = sc * e2;
        }
        const int lane = threadIdx.x & 63;
        const bool staged = n <= BATCH;  // the forward's only batch is still in s_rec
        if (in_lds)
            bwd_walk<NT, TexT, false, PIPE, LDSA>(n, [&](int j) { return s_ids[j]; }, staged, st, s_rec,
                                            s_grad,
                                      recs,
                                      atlas, Wp, zcell, tg, vmask, g0, g1, g2, 0.f, b0, b1,
                                      b2,
                                      tg.valid ? K : -1, TK, dparams, cu1, cv1, cu_cv2, cv_cu,
                                      lane);
        else
            bwd_walk<NT, TexT, false, PIPE, LDSA>(n, [&](int j) { return ((volatile int *)seg)[j]; },
                                      staged, Stored<1, TexT>(), s_rec, s_grad, recs, atlas, Wp, zcell, tg, vmask,
                                      g0,
                                      g1, g2,
                                      0.f, b0, b1, b2, tg.valid ? K : -1, TK, dparams, cu1, cv1,
                                      cu_cv2, cv_cu, lane);
        const float ws = wave_sum(sq);
        if (lane == 0) s_loss[threadIdx.x >> 6] = ws;
        __syncthreads();
        if (threadIdx.x == 0) {
            float t = 0.f;
            for (int w = 0; w < TS * TS / 64; ++w) t += s_loss[w];
            loss_tile[tile] = t;
        }
    }
    };
    run_schedule<PERSIST>(sched, grab, order, queue, n_tiles, tile_body);
}

// The backward's walk over a tile's sorted list (entry j's id is id_at(j)), back to front in
// batches of 64 entries (Supp. Eqs. S4-S5, Eq. 7): per pixel, g = dL/dI, ga = dL/dA, G = the
// background, and the forward's (K, T_K). `staged`: the whole list (n <= 64) is already in
// s_rec, staged by the forward of the fused step. The waves add their reduced partials into
// s_grad (LDS, one float per staged entry and parameter, zero on entry), which is flushed to
// dparams with one global atomic per (entry, parameter) after each batch: the tile's waves share
// one global add, and no global atomic is outstanding while a wave waits for its texels (on
// gfx950 the vector-memory counter retires in order, so a texel wait would also wait for the
// acknowledgement of every earlier atomic).
//
// The lanes sum only the factors that vary per pixel; the primitive's own constant factors are
// applied once per entry at the flush (the sums are linear in them):
//     s0 = sum dal MU,  s1 = sum dal MV      x, y:     -k_a (f_aU s0 + f_aV s1), -k_a (f_bU s0 + f_bV s1)
//     s2 = sum dal (MU U_c + MV V_c)         log s:    -k_a s2
//     s3 = sum dal (MU r V_c - MV U_c / r)   theta:    k_a s3
//     s4 = sum dal M                         nu:       k_a (1 - sigma) s4 (kaom)
//     s5..s7 = sum g_c T_j alpha_j           colours:  c (1 - c) s5..s7
// with dal = dL/dalpha_j, U_c, V_c the bitmap coordinates about the centre and r the ratio of the
// bitmap's half-extents. Each lane centres its coordinates (float64 subtraction, then the
// conversion): summing the uncentred coordinates and subtracting cu1 s0 + cv1 s1 at the flush
// instead saves two instructions but cancels, and it was measured to lose about two decimal
// digits on the angle's gradient.
template <int NT, typename TexT, bool HAS_GA, bool PIPE, bool LDSA, int TS, int SV,
          typename IdAt>
__device__ __forceinline__ void bwd_walk(int n, IdAt id_at, bool staged,
                                         const Stored<SV, TexT> &st,
                                         PrimRec *__restrict__ s_rec,
                                         float *__restrict__ s_grad,
                                         const PrimRec *__restrict__ recs,
                                         const TexT *__restrict__ atlas, int Wp, int zcell,
                                         const TileGeom<TS> &tg, uint64_t vmask, float g0,
                                         float g1, float g2, float ga, float G0, float G1,
                                         float G2, int K, float TK, float *__restrict__ dparams,
                                         double cu1, double cv1, float cu_cv2, float cv_cu,
                                         int lane)
{
    const double xd = tg.px, yd = tg.py;
    float Bk = 1.f, Trun = 0.f;  // behind K the transmittance is 0
    // g is fixed per pixel, so the walk carries only the projection gG = g . G of the composite
    // behind the current layer (G starts at the background and advances as G + alpha (c - G))
    float gG = fmaf(g2, G2, fmaf(g1, G1, g0 * G0));
    // Pipelined walk: the next staged entry (descending list order: back to front) that a lane
    // of this wave lies in, or -1; its cell is requested for every lane (for entry -1, and for
    // lanes outside the support, the all-zero cell), with the bitmap coordinates about the
    // centre that the geometric gradients use.
    auto find = [&](uint64_t &hits, Cell<TexT> &c, float &Uc, float &Vc) {
        int e = -1;
        double U = 0.0, V = 0.0;
        uint64_t msk = 0;
        while (hits) {
            const int k = 63 - __builtin_clzll(hits);
            hits ^= 1ull << k;
            const PrimRec &r = s_rec[k];
            U = fma(r.aU, xd, fma(r.bU, yd, r.eU));
            V = fma(r.aV, xd, fma(r.bV, yd, r.eV));
            msk = support_mask(r, U, V, vmask);
            if (msk != 0) { e = k; break; }
        }
        request_cell<TexT, true, LDSA>(c, atlas, e >= 0 ? s_rec[e].tex : 0, Wp, U, V,
                                       __builtin_amdgcn_inverse_ballot_w64(msk), zcell);
        Uc = (float)(U - cu1);
        Vc = (float)(V - cv1);
        return e;
    };
    // every lane runs the update; outside the support alpha = M = dM = 0, so its partials are
    // zero and its state (T, G, B) passes through unchanged (no branch and no zeroing: the
    // vector instructions issue for the whole wave either way)
    auto under_m = [&](int e, int j, float M, float MU, float MV, float Ub, float Vb) {
        const PrimRec &r = s_rec[e];
        const float4 kc = *reinterpret_cast<const float4 *>(&r.ka);  // ka, cr, cg, cb: one read
        float d[8];
        const float a = kc.x * M;
        const float m = 1.f - a;
        // T_j = T_{j+1} / (1 - alpha_j) with the hardware reciprocal (1 ulp). In front of K,
        // T_j (1 - alpha_j) >= TAU, so 1 - alpha_j > 0 and the reciprocal is finite. Behind K the
        // running value is 0, and the legacy multiply (0 times anything is 0) keeps it 0 where
        // alpha = 1 makes the reciprocal infinite.
        const float Tr = dbmp_mul_legacy(Trun, __builtin_amdgcn_rcpf(m));
        const float Tj = j == K ? TK : Tr;
        Trun = Tj;
        // g . (c_j - G): the colour's lead over the composite behind it, which also advances
        // g . G to the composite behind layer j - 1: g . (G + alpha (c - G))
        const float lead = fmaf(g2, kc.w, fmaf(g1, kc.z, fmaf(g0, kc.y, -gG)));
        float dal = lead;
        if (HAS_GA) dal = fmaf(ga, Bk, dal);
        dal *= Tj;
        const float ta = Tj * a;
        d[5] = g0 * ta;
        d[6] = g1 * ta;
        d[7] = g2 * ta;
        d[4] = dal * M;
        const float gU = dal * MU, gV = dal * MV;
        d[0] = gU;
        d[1] = gV;
        d[2] = fmaf(gU, Ub, gV * Vb);
        d[3] = fmaf(gU * cu_cv2, Vb, -(gV * Ub));  // times cv_cu at the flush
        gG = fmaf(a, lead, gG);
        Bk *= m;
        // lane 8q holds the wave total of value q; eight lanes add into the entry's LDS slots.
        // (Stopping the butterfly after the row mirror and letting all 64 lanes add their
        // partials, 8 lanes per address, saves 4 instructions but serialised in the LDS atomic
        // unit: it made the 2048^2 fit step's raster launch twice as long.)
        const float tot = reduce8(d, lane);
        asm volatile("" ::"v"(tot));  // formed on every lane: the last add stays fused with its DPP move
        if ((lane & 7) == 0)
            __hip_atomic_fetch_add(s_grad + e * 8 + (lane >> 3), tot, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    auto under = [&](int e, int j, const Cell<TexT> &c, float Ub, float Vb) {
        const Bil<TexT> b = blend<TexT>(c);
        under_m(e, j, b.m(), b.mu(), b.mv(), Ub, Vb);
    };
    for (int hi = n; hi > 0; hi -= BATCH) {
        const int b0 = max(0, hi - BATCH), cnt = hi - b0;
        if (!(staged && b0 == 0)) {
            __syncthreads();  // the previous batch is consumed
            stage_batch<NT>(s_rec, recs, b0, cnt, id_at);
            __syncthreads();
        }
        uint64_t hits = batch_hits(s_rec, cnt, tg.bx0, tg.by0);
        // entries up to the last stored visit were either stored or had no support lane: the
        // walk below takes the entries behind them, then the stored visits
        const bool use_st = staged && b0 == 0 && st.n > 0;
        if (use_st) hits &= st.last >= 63 ? 0ull : ~0ull << (st.last + 1);
        if constexpr (PIPE) {
            // two cells in turn: the next entry's texels are in flight while the current one's
            // gradient terms are formed (the last request of a batch is dropped)
            Cell<TexT> ca, cb;
            float ua, va, ub, vb;
            int ea = find(hits, ca, ua, va);
            while (ea >= 0) {
                const int eb = find(hits, cb, ub, vb);
                under(ea, b0 + ea, ca, ua, va);
                if (eb < 0) { drop_cell(cb); break; }
                ea = find(hits, ca, ua, va);
                under(eb, b0 + eb, cb, ub, vb);
            }
        } else {
            while (hits) {  // descending list order: back to front
                const int e = 63 - __builtin_clzll(hits);
                hits ^= 1ull << e;
                const PrimRec &r = s_rec[e];
                const double U = fma(r.aU, xd, fma(r.bU, yd, r.eU));
                const double V = fma(r.aV, xd, fma(r.bV, yd, r.eV));
                const uint64_t msk = support_mask(r, U, V, vmask);
                if (msk == 0) continue;
                Cell<TexT> c;
                request_cell<TexT, false, LDSA>(c, atlas, r.tex, Wp, U, V,
                                                __builtin_amdgcn_inverse_ballot_w64(msk), zcell);
                under(e, b0 + e, c, (float)(U - cu1), (float)(V - cv1));
            }
        }
        if (use_st) {  // the stored visits, back to front
#pragma unroll
            for (int v = SV - 1; v >= 0; --v) {
                if (v >= st.n) continue;
                const int e = st.e[v];
                const PrimRec &r = s_rec[e];
                const double U = fma(r.aU, xd, fma(r.bU, yd, r.eU));
                const double V = fma(r.aV, xd, fma(r.bV, yd, r.eV));
                under_m(e, b0 + e, st.b[v].m(), st.b[v].mu(), st.b[v].mv(), (float)(U - cu1),
                        (float)(V - cv1));
            }
        }
        // every wave has added its partials: one global atomic per (entry, parameter) per tile
        __syncthreads();
        for (int t = threadIdx.x; t < cnt * 8; t += NT) {
            // an entry's 8 slots lie in one wave, whose lanes read s0, s1 and their own slot
            // before any lane clears its slot (one instruction stream); then one atomic per lane
            const int q = t & 7;
            const PrimRec &r = s_rec[t >> 3];
            const float s0 = s_grad[t & ~7], s1 = s_grad[(t & ~7) + 1], v = s_grad[t];
            float x;
            if (q < 2)
                x = -r.ka * fmaf(q == 0 ? r.faU : r.fbU, s0, (q == 0 ? r.faV : r.fbV) * s1);
            else
                x = (q == 2 ? -r.ka : q == 3 ? r.ka * cv_cu : q == 4 ? r.kaom : q == 5 ? r.ccr
                     : q == 6 ? r.ccg : r.ccb) * v;
            s_grad[t] = 0.f;  // ready for the next batch
            if (x != 0.f) unsafeAtomicAdd(dparams + (size_t)r.id * 8 + q, x);
        }
    }
}

// MSE: the backward forms dL/dI = scale (I - target) itself from the forward's image and writes
// the workgroup's sum of squared differences to loss_tile[tile] (reduced on request).
template <int TS, typename TexT, bool BG_PP, bool HAS_GA, bool MSE, int LAUNCH>
__global__ void __launch_bounds__(TS * TS)
k_raster_bwd(const PrimRec *__restrict__ recs, const int *__restrict__ lists, int list_cap,
             const int *__restrict__ tile_len,
             const ImgDev *__restrict__ imgs, int n_images, int n_tiles,
             const TexT *__restrict__ atlas_g, int Wp, int zcell, const float *__restrict__ bg,
             const int *__restrict__ saveK, const float *__restrict__ saveT,
             const float *__restrict__ gI, const float *__restrict__ target,
             float *__restrict__ loss_tile, const float *__restrict__ gA,
             float *__restrict__ dparams, double cu1, double cv1, float cu_cv2, float cv_cu,
             const int *__restrict__ flags, int sched, int grab,
             const int *__restrict__ order, int *__restrict__ queue, int atl_bytes)
{
    constexpr bool LDSA = LAUNCH == LAUNCH_TILE_PIPE_LDS;
    constexpr bool PERSIST = LAUNCH == LAUNCH_PERSISTENT;
    constexpr bool PIPE = LAUNCH == LAUNCH_TILE_PIPE || LDSA;
    __shared__ PrimRec s_rec[BATCH];
    __shared__ float s_loss[TS * TS / 64];
    __shared__ float s_grad[BATCH * 8];  // per-entry partial sums of the gradient
    for (int i = threadIdx.x; i < BATCH * 8; i += TS * TS) s_grad[i] = 0.f;
    __syncthreads();
    const TexT *atlas = atlas_g;
    if constexpr (LDSA) atlas = stage_atlas<TexT>(atlas_g, atl_bytes);
    auto tile_body = [&](const int tile) {
        const int n = tile_len[tile];
        if (n > list_cap) return;  // the forward did not render this tile
        const TileGeom<TS> tg = tile_geom<TS>(tile, imgs, n_images);
        const int lane = threadIdx.x & 63;
        const ImgDev &D = tg.D;
        const double xd = tg.px, yd = tg.py;
        const uint64_t vmask = __ballot(tg.valid);
        const size_t plane = (size_t)D.H * D.W;
        const long long gp = D.pix_off + tg.pix;
        float g0 = 0.f, g1 = 0.f, g2 = 0.f, ga = 0.f, G0 = 0.f, G1 = 0.f, G2 = 0.f, TK = 0.f;
        float sq = 0.f;
        int K = -1;
        if (tg.valid) {
            const float *gp3 = gI + 3 * D.pix_off + tg.pix;  // MSE: the forward's image
            g0 = gp3[0]; g1 = gp3[plane]; g2 = gp3[2 * plane];
            if (MSE) {
                const float *tp = target + 3 * D.pix_off + tg.pix;
                const float e0 = g0 - tp[0], e1 = g1 - tp[plane], e2 = g2 - tp[2 * plane];
                sq = fmaf(e0, e0, fmaf(e1, e1, e2 * e2));
                const float sc = 2.f / (3.f * (float)plane);  // mean over the image's 3HW values
                g0 = sc * e0; g1 = sc * e1; g2 = sc * e2;
            }
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
        const int *seg = lists + (size_t)tile * list_cap;
        bwd_walk<TS * TS, TexT, HAS_GA, PIPE, LDSA>(n, [&](int j) { return seg[j]; }, false,
                                              Stored<1, TexT>(), s_rec,
                                              s_grad,
                                        recs,
                                        atlas, Wp, zcell, tg, vmask, g0, g1, g2, ga, G0, G1, G2,
                                        K, TK,
                                        dparams, cu1, cv1, cu_cv2, cv_cu, lane);
        if (MSE) {
            const float ws = wave_sum(sq);
            if (lane == 0) s_loss[threadIdx.x >> 6] = ws;
            __syncthreads();
            if (threadIdx.x == 0) {
                float t = 0.f;
                for (int w = 0; w < TS * TS / 64; ++w) t += s_loss[w];
                loss_tile[tile] = t;
            }
        }
    };
    run_schedule<PERSIST>(sched, grab, order, queue, n_tiles, tile_body);
}

// ------------------------------------------------------------------------------------------
// Host side: launch of one kernel build (LAUNCH as above), dispatched over the runtime choices
// ------------------------------------------------------------------------------------------
// The pipelined walks pay off where the launch leaves SIMDs with few waves: at most 4 waves per
// SIMD (16 per compute unit) across the one-tile-per-workgroup grid.
static inline bool pipelined(const RasterArgs &a)
{
    const long long waves = (long long)a.n_tiles * (a.TS * a.TS / 64);
    return a.sched != SCHED_PERSISTENT && waves <= 16LL * a.n_cu;
}

// Launches `kern`; with timing events armed, through hipExtLaunchKernel, which has the device
// record them when the kernel starts and when it ends.
template <typename K, typename... Args>
static void launch_kernel(K kern, int grid, int block, size_t lds, hipStream_t st,
                          hipEvent_t e0, hipEvent_t e1, Args... args)
{
    if (e0 && e1)
        hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, st, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, st, args...);
}

// Workgroups of a kernel that one compute unit holds at once (registers and LDS permitting).
// A persistent grid larger than what is resident would leave its surplus workgroups waiting
// for others to finish, and their whole share of the tiles would run after them.
template <typename K>
static int resident_per_cu(K kern, int threads)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, threads, 0) != hipSuccess || n < 1)
        n = 1;
    return n;
}

// The persistent grid: the schedule's workgroups per compute unit, at most what is resident.
template <typename K>
static int persistent_grid(K kern, int threads, const RasterArgs &a)
{
    static const int resident = resident_per_cu(kern, threads);
    return std::min(std::min(a.grid, a.n_cu * resident), a.n_tiles);
}

template <int TS, typename TexT, bool BGPP, bool FUSED, int LAUNCH>
static void fwd_t(const RasterArgs &a, hipStream_t st)
{
    const double cu = 0.5 * (a.Wb - 1), cv = 0.5 * (a.Hb - 1);
    const int grid = LAUNCH == LAUNCH_PERSISTENT
                         ? persistent_grid(k_raster_fwd<TS, TexT, BGPP, FUSED, LAUNCH>, TS * TS, a)
                         : a.n_tiles;
    const int atl = LAUNCH == LAUNCH_TILE_PIPE_LDS ? a.atlas_lds_bytes : 0;
    launch_kernel(k_raster_fwd<TS, TexT, BGPP, FUSED, LAUNCH>, grid, TS * TS,
        (size_t)((atl + 15) & ~15), st, a.ev_start, a.ev_stop, a.recs, const_cast<int *>(a.lists), a.list_cap, a.tile_count, a.tile_len,
        a.list_max, a.imgs,
        a.n_images, a.n_tiles, (const TexT *)a.atlas_pad, a.Wp, a.zcell, a.bg, a.image, a.alpha,
        a.saveK,
        a.saveT, a.flags, a.pair_counter, a.sched, a.grab, a.order, a.queue, a.target,
        a.loss_tile, a.dparams, cu + 1.0, cv + 1.0, (float)((cu / cv) * (cu / cv)),
        (float)(cv / cu),
        a.fit_state, atl);
}

template <int TS, typename TexT, bool BGPP, bool GA, bool MSE, int LAUNCH>
static void bwd_t(const RasterArgs &a, hipStream_t st)
{
    const double cu = 0.5 * (a.Wb - 1), cv = 0.5 * (a.Hb - 1);
    const int grid = LAUNCH == LAUNCH_PERSISTENT
                         ? persistent_grid(k_raster_bwd<TS, TexT, BGPP, GA, MSE, LAUNCH>, TS * TS, a)
                         : a.n_tiles;
    const int atl = LAUNCH == LAUNCH_TILE_PIPE_LDS ? a.atlas_lds_bytes : 0;
    launch_kernel(k_raster_bwd<TS, TexT, BGPP, GA, MSE, LAUNCH>, grid, TS * TS,
        (size_t)((atl + 15) & ~15), st, a.ev_start, a.ev_stop, a.recs, a.lists, a.list_cap, a.tile_len, a.imgs, a.n_images, a.n_tiles,
        (const TexT *)a.atlas_pad, a.Wp, a.zcell, a.bg, a.saveK, a.saveT, MSE ? a.image : a.gI,
        a.target,
        a.loss_tile, a.gA, a.dparams, cu + 1.0, cv + 1.0, (float)((cu / cv) * (cu / cv)),
        (float)(cv / cu), a.flags, a.sched, a.grab, a.order, a.queue + 2, atl);
}

template <int TS, typename TexT, int LAUNCH>
static void fwd_d1(const RasterArgs &a, hipStream_t st)
{
    if (a.target) {
        if (a.bg_pp) fwd_t<TS, TexT, true, true, LAUNCH>(a, st);
        else fwd_t<TS, TexT, false, true, LAUNCH>(a, st);
    } else {
        if (a.bg_pp) fwd_t<TS, TexT, true, false, LAUNCH>(a, st);
        else fwd_t<TS, TexT, false, false, LAUNCH>(a, st);
    }
}
template <int TS, int LAUNCH>
static void fwd_d0(const RasterArgs &a, hipStream_t st)
{
    if (a.dtype == 0) fwd_d1<TS, float, LAUNCH>(a, st); else fwd_d1<TS, uint16_t, LAUNCH>(a, st);
}
template <int LAUNCH>
static void raster_fwd_build(const RasterArgs &a, hipStream_t st)
{
    switch (a.TS) {
    case 8: fwd_d0<8, LAUNCH>(a, st); break;
    case 16: fwd_d0<16, LAUNCH>(a, st); break;
    default: fwd_d0<32, LAUNCH>(a, st); break;
    }
}

template <int TS, typename TexT, bool BGPP, bool GA, int LAUNCH>
static void bwd_d3(const RasterArgs &a, hipStream_t st)
{
    if (a.target) bwd_t<TS, TexT, BGPP, GA, true, LAUNCH>(a, st);
    else bwd_t<TS, TexT, BGPP, GA, false, LAUNCH>(a, st);
}
template <int TS, typename TexT, bool BGPP, int LAUNCH>
static void bwd_d2(const RasterArgs &a, hipStream_t st)
{
    if (a.gA) bwd_d3<TS, TexT, BGPP, true, LAUNCH>(a, st);
    else bwd_d3<TS, TexT, BGPP, false, LAUNCH>(a, st);
}
template <int TS, typename TexT, int LAUNCH>
static void bwd_d1(const RasterArgs &a, hipStream_t st)
{
    if (a.bg_pp) bwd_d2<TS, TexT, true, LAUNCH>(a, st);
    else bwd_d2<TS, TexT, false, LAUNCH>(a, st);
}
template <int TS, int LAUNCH>
static void bwd_d0(const RasterArgs &a, hipStream_t st)
{
    if (a.dtype == 0) bwd_d1<TS, float, LAUNCH>(a, st); else bwd_d1<TS, uint16_t, LAUNCH>(a, st);
}
template <int LAUNCH>
static void raster_bwd_build(const RasterArgs &a, hipStream_t st)
{
    switch (a.TS) {
    case 8: bwd_d0<8, LAUNCH>(a, st); break;
    case 16: bwd_d0<16, LAUNCH>(a, st); break;
    default: bwd_d0<32, LAUNCH>(a, st); break;
    }
}

}  // namespace dbmp
