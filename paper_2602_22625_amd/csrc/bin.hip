// Per-primitive setup and screen-tile binning (Sec. 3.1.1 "Parallelization": each primitive is
// assigned to every T x T tile its footprint overlaps; lists are composited front to back).
//
// Stages, all on the device and all asynchronous:
//   k_setup    pads every bitmap with a one-texel zero border (the zero padding of the bilinear
//              sampler) and finds each bitmap's tight non-zero box (once per atlas);
//   k_prep     per primitive: sigmoid/exp/sincos, the inverse affine map of Eqs. (1)-(2) folded
//              into U' = aU x + bU y + eU (float64), the exact support parallelogram and its
//              tile span; then the workgroup deals the (primitive, tile) pairs of its spans
//              over all its lanes, tests each tile (a separating-axis test, so rotated
//              primitives are not charged for the corners of their bounding box) and appends
//              the primitive's row to the tile's list.
// Every tile owns a list of fixed capacity (lists[t * cap .. ]), so appending needs one atomic
// per (tile, primitive) pair and no prefix scan or second pass; a tile whose list would
// overflow raises a flag and the caller grows the capacity. The forward raster kernel sorts
// each tile's list front to back (depth order = index order).
#include "dbmp_internal.h"

#include <limits.h>

namespace dbmp {

// ------------------------------------------------------------------------------------------
// k_setup
// ------------------------------------------------------------------------------------------
#define SETUP_THREADS 1024
#define SETUP_BATCH 8

template <typename TexT>
__global__ void __launch_bounds__(SETUP_THREADS)
k_setup(const TexT *__restrict__ atlas, int B, int Hb, int Wb, TexT *__restrict__ pad, int Wp,
        int *__restrict__ box)
{
    const int Hp = Hb + 2;
    if (blockIdx.x == 0)  // the two zero rows after the last bitmap (the all-zero cell)
        for (int i = threadIdx.x; i < 2 * Wp; i += SETUP_THREADS)
            pad[(size_t)B * Hp * Wp + i] = TexT(0);
    {
        const int b = blockIdx.x;
        const TexT *src = atlas + (size_t)b * Hb * Wb;
        TexT *dst = pad + (size_t)b * Hp * Wp;
        int xlo = INT_MAX, xhi = INT_MIN, ylo = INT_MAX, yhi = INT_MIN, bad = 0;
        const int total = Hp * Wp;
        for (int base = 0; base < total; base += SETUP_THREADS * SETUP_BATCH) {
            TexT v[SETUP_BATCH];
            int rr[SETUP_BATCH], cc[SETUP_BATCH];
#pragma unroll
            for (int q = 0; q < SETUP_BATCH; ++q) {  // issue every load of the batch first
                const int i = base + q * SETUP_THREADS + threadIdx.x;
                rr[q] = i / Wp - 1;
                cc[q] = i % Wp - 1;
                const bool inside = i < total && rr[q] >= 0 && rr[q] < Hb && cc[q] >= 0 &&
                                    cc[q] < Wb;
                v[q] = inside ? src[(size_t)rr[q] * Wb + cc[q]] : TexT(0);
            }
#pragma unroll
            for (int q = 0; q < SETUP_BATCH; ++q) {
                const int i = base + q * SETUP_THREADS + threadIdx.x;
                if (i >= total) continue;
                const float f = texel<TexT>(v[q]);
                if (!isfinite(f)) { bad = 1; v[q] = TexT(0); }
                if (f != 0.0f && isfinite(f)) {
                    xlo = min(xlo, cc[q]); xhi = max(xhi, cc[q]);
                    ylo = min(ylo, rr[q]); yhi = max(yhi, rr[q]);
                }
                dst[i] = v[q];
            }
        }
        __shared__ int s[5];
        if (threadIdx.x == 0) {
            s[0] = INT_MAX; s[1] = INT_MIN; s[2] = INT_MAX; s[3] = INT_MIN; s[4] = 0;
        }
        __syncthreads();
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            xlo = min(xlo, __shfl_xor(xlo, o)); xhi = max(xhi, __shfl_xor(xhi, o));
            ylo = min(ylo, __shfl_xor(ylo, o)); yhi = max(yhi, __shfl_xor(yhi, o));
        }
        if ((threadIdx.x & 63) == 0 && xlo <= xhi) {
            atomicMin(&s[0], xlo); atomicMax(&s[1], xhi);
            atomicMin(&s[2], ylo); atomicMax(&s[3], yhi);
        }
        if (bad) s[4] = 1;
        __syncthreads();
        if (threadIdx.x == 0) {
            // a bitmap holding a non-finite texel is marked; primitives using it raise the flag
            box[4 * b + 0] = s[4] ? INT_MIN : s[0]; box[4 * b + 1] = s[1];
            box[4 * b + 2] = s[2]; box[4 * b + 3] = s[3];
        }
    }
}

// ------------------------------------------------------------------------------------------
// Separating-axis test of the support parallelogram against a tile's pixel centres. U' and V'
// are affine in (x, y), so their range over the tile rectangle is attained at its corners; the
// tile's own axes are covered by the bounding-box span. The margin keeps the test conservative
// against rounding; the raster kernels test every pixel exactly.
// ------------------------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ bool tile_hits(const R &r, int X0, int X1, int Y0, int Y1)
{
    const double m = 1e-6;
    const double ux0 = r.aU * X0, ux1 = r.aU * X1, uy0 = r.bU * Y0, uy1 = r.bU * Y1;
    const double umin = r.eU + fmin(ux0, ux1) + fmin(uy0, uy1);
    const double umax = r.eU + fmax(ux0, ux1) + fmax(uy0, uy1);
    if (umax < r.Ulo - m || umin >= r.Uhi + m) return false;
    const double vx0 = r.aV * X0, vx1 = r.aV * X1, vy0 = r.bV * Y0, vy1 = r.bV * Y1;
    const double vmin = r.eV + fmin(vx0, vx1) + fmin(vy0, vy1);
    const double vmax = r.eV + fmax(vx0, vx1) + fmax(vy0, vy1);
    if (vmax < r.Vlo - m || vmin >= r.Vhi + m) return false;
    return true;
}

// ------------------------------------------------------------------------------------------
// Tiles by decreasing list length, for the sorted and persistent schedules: a histogram of the
// lengths (capped at ORDER_BINS - 1) in LDS, an exclusive scan of the bins from the longest
// down, then a scatter. Ties are placed in any order: every tile is computed independently, so
// the order changes no image bit. Run by NTH threads of one workgroup: by an extra workgroup of
// k_prep on the previous forward's lengths (small canvases: no launch of its own, and off the
// critical path), else by the many-workgroup form below after the binning.
// ------------------------------------------------------------------------------------------
constexpr int ORDER_BINS = 1024;
constexpr int ORDER_IN_PREP_MAX = 4096;  // tiles up to which the binning orders them
constexpr int ORDER_KEEP = 16;           // tile lengths per thread read once and kept

template <int NTH, bool ATOMIC_READS>
__device__ __forceinline__ void order_tiles(const int *__restrict__ tile_count, int n_tiles,
                                            int *__restrict__ order, int *hist, int *wsum)
{
    static_assert(ORDER_BINS % NTH == 0 && NTH % 64 == 0, "bins per thread");
    constexpr int BPT = ORDER_BINS / NTH;  // consecutive bins owned by one thread
    const int t = threadIdx.x;
    // bin 0 holds the longest lists
    auto bin = [](int len) { return ORDER_BINS - 1 - min(max(len, 0), ORDER_BINS - 1); };
    auto count = [&](int i) {
        // counts appended by other workgroups of the same launch are read at device scope
        return ATOMIC_READS ? __hip_atomic_load(tile_count + i, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT)
                            : tile_count[i];
    };
    // each thread's tiles' bins, read once (up to ORDER_KEEP per thread kept in registers)
    constexpr int KEEP = ORDER_KEEP;
    int kb[KEEP];
#pragma unroll
    for (int k = 0; k < KEEP; ++k) {
        const int i = t + k * NTH;
        kb[k] = i < n_tiles ? bin(count(i)) : 0;
    }
    for (int b = t; b < ORDER_BINS; b += NTH) hist[b] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KEEP; ++k)
        if (t + k * NTH < n_tiles) atomicAdd(&hist[kb[k]], 1);
    for (int i = t + KEEP * NTH; i < n_tiles; i += NTH) atomicAdd(&hist[bin(count(i))], 1);
    __syncthreads();
    // exclusive scan: within the thread's bins, then wave-inclusive scans of the thread sums,
    // then the wave totals
    int sum = 0;
    for (int k = 0; k < BPT; ++k) {
        const int v = hist[t * BPT + k];
        hist[t * BPT + k] = sum;
        sum += v;
    }
    int x = sum;
    const int lane = t & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[t >> 6] = x;
    __syncthreads();
    int base = x - sum;
    for (int w = 0; w < (t >> 6); ++w) base += wsum[w];
    for (int k = 0; k < BPT; ++k) hist[t * BPT + k] += base;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KEEP; ++k) {
        const int i = t + k * NTH;
        if (i < n_tiles) order[atomicAdd(&hist[kb[k]], 1)] = i;
    }
    for (int i = t + KEEP * NTH; i < n_tiles; i += NTH) {
        const int pos = atomicAdd(&hist[bin(count(i))], 1);
        order[pos] = i;
    }
}

// Many tiles (beyond the binning's own ordering): the same counting sort spread over
// workgroups of ORDER_CHUNK tiles, so that no single compute unit takes every tile's LDS atomic
// (most tiles fall into a few length bins, whose same-address atomics serialise). Three
// launches: per-workgroup histograms (hist[group * ORDER_BINS + bin]); one exclusive scan over
// them in bin-major order, longest bin first; then each workgroup places its tiles at its
// offsets.
constexpr int ORDER_CHUNK = 2048;
constexpr int ORDER_THREADS = 256;

size_t order_hist_bytes(long long n_tiles)
{
    return 4 * (size_t)ORDER_BINS * (size_t)((n_tiles + ORDER_CHUNK - 1) / ORDER_CHUNK);
}

__device__ __forceinline__ int order_bin(int len)
{
    return ORDER_BINS - 1 - min(max(len, 0), ORDER_BINS - 1);  // bin 0: the longest lists
}

__global__ void __launch_bounds__(ORDER_THREADS)
k_order_count(const int *__restrict__ tile_count, int n_tiles, int *__restrict__ ghist)
{
    __shared__ int hist[ORDER_BINS];
    const int t0 = blockIdx.x * ORDER_CHUNK;
    for (int b = threadIdx.x; b < ORDER_BINS; b += ORDER_THREADS) hist[b] = 0;
    __syncthreads();
    for (int i = t0 + threadIdx.x; i < min(t0 + ORDER_CHUNK, n_tiles); i += ORDER_THREADS)
        atomicAdd(&hist[order_bin(tile_count[i])], 1);
    __syncthreads();
    for (int b = threadIdx.x; b < ORDER_BINS; b += ORDER_THREADS)
        ghist[(size_t)blockIdx.x * ORDER_BINS + b] = hist[b];
}

// One workgroup of ORDER_BINS threads: thread b owns bin b's counts of the G groups (a wave reads
// one group's consecutive bins), takes their total, adds the exclusive sum of the earlier bins
// (wave scans of the totals), and writes its groups' offsets. The counts are read ORDER_IN_FLIGHT
// at a time, so their loads overlap.
constexpr int ORDER_IN_FLIGHT = 32;

__global__ void __launch_bounds__(ORDER_BINS) k_order_scan(int *__restrict__ ghist, int G)
{
    __shared__ int wsum[ORDER_BINS / 64];
    const int b = threadIdx.x, lane = b & 63;
    int sum = 0;
    for (int g0 = 0; g0 < G; g0 += ORDER_IN_FLIGHT) {
        int v[ORDER_IN_FLIGHT];
#pragma unroll
        for (int k = 0; k < ORDER_IN_FLIGHT; ++k)
            v[k] = g0 + k < G ? ghist[(size_t)(g0 + k) * ORDER_BINS + b] : 0;
#pragma unroll
        for (int k = 0; k < ORDER_IN_FLIGHT; ++k) sum += v[k];
    }
    int x = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[b >> 6] = x;
    __syncthreads();
    int run = x - sum;
    for (int w = 0; w < (b >> 6); ++w) run += wsum[w];
    for (int g0 = 0; g0 < G; g0 += ORDER_IN_FLIGHT) {
        int v[ORDER_IN_FLIGHT];
#pragma unroll
        for (int k = 0; k < ORDER_IN_FLIGHT; ++k)
            v[k] = g0 + k < G ? ghist[(size_t)(g0 + k) * ORDER_BINS + b] : 0;
#pragma unroll
        for (int k = 0; k < ORDER_IN_FLIGHT; ++k) {
            if (g0 + k < G) ghist[(size_t)(g0 + k) * ORDER_BINS + b] = run;
            run += v[k];
        }
    }
}

__global__ void __launch_bounds__(ORDER_THREADS)
k_order_place(const int *__restrict__ tile_count, int n_tiles, const int *__restrict__ ghist,
              int *__restrict__ order)
{
    __shared__ int pos[ORDER_BINS];
    const int t0 = blockIdx.x * ORDER_CHUNK;
    for (int b = threadIdx.x; b < ORDER_BINS; b += ORDER_THREADS)
        pos[b] = ghist[(size_t)blockIdx.x * ORDER_BINS + b];
    __syncthreads();
    for (int i = t0 + threadIdx.x; i < min(t0 + ORDER_CHUNK, n_tiles); i += ORDER_THREADS)
        order[atomicAdd(&pos[order_bin(tile_count[i])], 1)] = i;
}

// ------------------------------------------------------------------------------------------
// k_prep
// ------------------------------------------------------------------------------------------
#define PREP_THREADS 256
// Primitives per workgroup (PP): PP lanes of the first wave compute records, all lanes walk
// tiles. 16 for small primitive counts (more workgroups in flight), 64 for large ones (a quarter
// of the workgroups, each with as short a critical path).
constexpr int PREP_SMALL_N = 16384;

// The fields of a record the tile walk needs, kept in LDS between the two phases of k_prep.
struct WalkRec {
    double aU, bU, eU, aV, bV, eV, Ulo, Uhi, Vlo, Vhi;
    int tx0, tx1, ty0, ty1, tile_off, ntx, W, H;
};

template <int PREP_PRIMS>
__global__ void __launch_bounds__(PREP_THREADS)
k_prep(const float *params, const int *__restrict__ idx, long long n_rows,
       const ImgDev *__restrict__ imgs, int n_images, const int *__restrict__ box, int B, int Hb,
       int Wb, int Wp, float alpha_max, int TS, PrimRec *__restrict__ recs,
       int *__restrict__ tile_count, int *__restrict__ lists, int list_cap,
       int *__restrict__ flags, int n_tiles, int *__restrict__ order,
       const int *__restrict__ prev_len, AdamArgs adam)
{
    if (order && blockIdx.x == gridDim.x - 1) {
        // the extra workgroup: tiles by decreasing list length of the previous forward, while
        // the others bin (any permutation is a valid order; a fit's lists change slowly)
        __shared__ int hist[ORDER_BINS];
        __shared__ int wsum[PREP_THREADS / 64];
        order_tiles<PREP_THREADS, false>(prev_len, n_tiles, order, hist, wsum);
        return;
    }
    __shared__ WalkRec s_rec[PREP_PRIMS];
    __shared__ int s_span[PREP_PRIMS + 1];  // exclusive prefix sums of the tile spans, then the total
    int span = 0;                           // this record lane's primitive: tiles in its span
    // a fit step's pending Adam update (wave-uniform: every workgroup reads the same flag)
    const bool adam_on = adam.params && adam.state[2] != 0;
    const int t_adam = adam_on ? adam.state[0] + 1 : 0;
    // The parameter-wise work is spread over the LANES = PREP_THREADS / PREP_PRIMS lanes of each
    // primitive (16 or 4) before one lane per primitive assembles the record: the lanes take the
    // 8 parameters' Adam updates in turn, then the 9 float64 exponentials and the sine and
    // cosine. Every lane of a pass runs the same instructions, so a pass costs one evaluation,
    // and a wave's loads of parameters and moments are coalesced. The values are those of a
    // one-lane evaluation; the update is k_adam's (zero_grad), bit for bit.
    // The record lane's image record, bitmap index and bitmap box, requested before the
    // parameter-wise passes so that their latency overlaps them.
    const long long g_rec = (long long)blockIdx.x * PREP_PRIMS + threadIdx.x;
    int b = 0, k = 0, xlo = 0, xhi = -1, ylo = 0, yhi = -1;
    bool k_ok = false;
    ImgDev D{};
    if (threadIdx.x < PREP_PRIMS && g_rec < n_rows) {
        b = find_by_prim(imgs, n_images, g_rec);
        D = imgs[b];
        k = idx[g_rec];
        k_ok = k >= 0 && k < B;
        if (k_ok) {
            xlo = box[4 * k];
            xhi = box[4 * k + 1];
            ylo = box[4 * k + 2];
            yhi = box[4 * k + 3];
        }
    }
    constexpr int LANES = PREP_THREADS / PREP_PRIMS;
    constexpr int PPL = (8 + LANES - 1) / LANES;  // parameters per lane
    static_assert(LANES >= 4 && PREP_THREADS % PREP_PRIMS == 0, "lanes per primitive");
    __shared__ float s_p[PREP_PRIMS * 8];     // parameters after the update
    __shared__ double s_e[PREP_PRIMS * 12];   // exponentials, sine, cosine
    {
        const int pl = threadIdx.x / LANES, l = threadIdx.x % LANES;
        const long long gq = (long long)blockIdx.x * PREP_PRIMS + pl;
        // all loads first, then the arithmetic, then the stores (the buffers are distinct, but
        // the compiler cannot know it, and would otherwise wait for each store)
        float pq[PPL], gv[PPL], mv[PPL], vv[PPL];
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            const int q = l + k * LANES;
            if (gq < n_rows && q < 8) {
                pq[k] = params[gq * 8 + q];
                // read whenever the update buffers are given, used only if an update is
                // pending: the loads then overlap the load of the pending flag
                if (adam.params) {
                    gv[k] = adam.grad[gq * 8 + q];
                    mv[k] = adam.m[gq * 8 + q];
                    vv[k] = adam.v[gq * 8 + q];
                }
            }
        }
        if (adam_on) {
            const float c1 = (float)(1.0 - pow((double)adam.b1, (double)t_adam));
            const float c2 = (float)(1.0 - pow((double)adam.b2, (double)t_adam));
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                const int q = l + k * LANES;
                if (gq < n_rows && q < 8) {
                    const float gi = gv[k];
                    mv[k] = fmaf(adam.b1, mv[k], (1.f - adam.b1) * gi);
                    vv[k] = fmaf(adam.b2, vv[k], (1.f - adam.b2) * gi * gi);
                    const float mhat = mv[k] / c1, vhat = vv[k] / c2;
                    pq[k] = pq[k] - adam.lr * mhat / (sqrtf(vhat) + adam.eps);
                }
            }
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                const int q = l + k * LANES;
                if (gq < n_rows && q < 8) {
                    adam.grad[gq * 8 + q] = 0.f;
                    adam.m[gq * 8 + q] = mv[k];
                    adam.v[gq * 8 + q] = vv[k];
                    adam.params[gq * 8 + q] = pq[k];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
            const int q = l + k * LANES;
            if (gq < n_rows && q < 8) s_p[pl * 8 + q] = pq[k];
        }
        __syncthreads();
        if (gq < n_rows) {
            // item q: s = exp(p2); 1/(1 + exp(-p4)) and 1/(1 + exp(p4)); 1/(1 + exp(-p5..7));
            // exp(p5..7) (the colour derivative divides by 1 + exp(p)); item 9: sin, cos of p3
            const float *pp = s_p + pl * 8;
            for (int q = l; q < 10; q += LANES) {
                if (q < 9) {
                    const double x = q == 0 ? (double)pp[2]
                                   : q == 1 ? -(double)pp[4]
                                   : q == 2 ? (double)pp[4]
                                   : q < 6 ? -(double)pp[2 + q]
                                           : (double)pp[q - 1];
                    const double e = exp(x);
                    s_e[pl * 12 + q] = (q == 0 || q >= 6) ? e : 1.0 / (1.0 + e);
                } else {
                    double st, ct;
                    sincos((double)pp[3], &st, &ct);
                    s_e[pl * 12 + 9] = st;
                    s_e[pl * 12 + 10] = ct;
                }
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < PREP_PRIMS) {
        const long long g = (long long)blockIdx.x * PREP_PRIMS + threadIdx.x;
        PrimRec rec;
        rec.aU = rec.bU = rec.eU = rec.aV = rec.bV = rec.eV = 0.0;
        rec.Ulo = 1.0; rec.Uhi = 0.0; rec.Vlo = 1.0; rec.Vhi = 0.0;  // empty support
        rec.ka = 0.f; rec.cr = rec.cg = rec.cb = 0.f; rec.tex = 0; rec.kaom = 0.f;
        rec.ccr = rec.ccg = rec.ccb = 0.f;
        rec.faU = rec.fbU = rec.faV = rec.fbV = 0.f;
        int tx0 = 1, tx1 = 0, ty0 = 1, ty1 = 0;  // tile span of the pixel box (empty)
        rec.px0 = 1; rec.px1 = 0; rec.py0 = 1; rec.py1 = 0;
        rec.id = (int)g;
        rec.pad[0] = rec.pad[1] = 0;
        WalkRec &wr = s_rec[threadIdx.x];
        wr.tile_off = wr.ntx = wr.W = wr.H = 0;
        if (g < n_rows) {
            // s = exp(p2); sin, cos of p3; the sigmoid of the opacity logit and its complement;
            // the colour sigmoids and exp of the colour logits
            float p[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) p[j] = s_p[threadIdx.x * 8 + j];
            const double *e = s_e + threadIdx.x * 12;
            const double s = e[0], sig = e[1], omsig = e[2], st = e[9], ct = e[10];
            const double c3[3] = {e[3], e[4], e[5]}, ep[3] = {e[6], e[7], e[8]};
            wr.tile_off = D.tile_off; wr.ntx = D.ntx; wr.W = D.W; wr.H = D.H;
            if (g >= D.prim_off && g < D.prim_off + D.N) {
                bool ok = true;
                if (!k_ok) {
                    atomicOr(&flags[F_S_BADIDX], 1);
                    ok = false;
                }
                bool fin = true;
#pragma unroll
                for (int j = 0; j < 8; ++j) fin = fin && isfinite(p[j]);
                if (!(s > 0.0) || !isfinite(s)) fin = false;  // scale underflows or overflows
                if (!fin) {
                    atomicOr(&flags[F_S_NONFINITE], 1);
                    ok = false;
                }
                if (ok) {
                    const double inv_s = 1.0 / s;
                    const double cu = 0.5 * (Wb - 1), cv = 0.5 * (Hb - 1);  // dU/du, dV/dv
                    const double x = p[0], y = p[1];
                    // Eq. (1)-(2): u = (ct dx + st dy)/s, v = (-st dx + ct dy)/s, U = cu (u + 1),
                    // plus the one-texel shift into the padded bitmap.
                    rec.aU = cu * ct * inv_s;  rec.bU = cu * st * inv_s;
                    rec.aV = -cv * st * inv_s; rec.bV = cv * ct * inv_s;
                    rec.eU = (cu + 1.0) - rec.aU * x - rec.bU * y;
                    rec.eV = (cv + 1.0) - rec.aV * x - rec.bV * y;
                    rec.faU = (float)rec.aU; rec.fbU = (float)rec.bU;
                    rec.faV = (float)rec.aV; rec.fbV = (float)rec.bV;
                    rec.ka = (float)(alpha_max * sig);
                    rec.kaom = (float)(alpha_max * sig * omsig);
                    rec.cr = (float)c3[0]; rec.cg = (float)c3[1]; rec.cb = (float)c3[2];
                    rec.ccr = (float)(c3[0] / (1.0 + ep[0]));  // c (1 - c)
                    rec.ccg = (float)(c3[1] / (1.0 + ep[1]));
                    rec.ccb = (float)(c3[2] / (1.0 + ep[2]));
                    const int Hp = Hb + 2;
                    rec.tex = k * Hp * Wp;
                    if (xlo == INT_MIN) {  // the bitmap holds a non-finite texel (read as 0)
                        atomicOr(&flags[F_S_NONFINITE], 1);
                        xlo = 0;
                    }
                    if (xlo <= xhi) {
                        // floor(U') in [xlo, xhi + 1] reads at least one non-zero texel (padded
                        // columns xlo + 1 .. xhi + 1); elsewhere M and its derivatives are 0.
                        rec.Ulo = xlo; rec.Uhi = xhi + 2;
                        rec.Vlo = ylo; rec.Vhi = yhi + 2;
                        double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            const double Uc = (c & 1) ? rec.Uhi : rec.Ulo;
                            const double Vc = (c & 2) ? rec.Vhi : rec.Vlo;
                            const double u = (Uc - 1.0) / cu - 1.0, v = (Vc - 1.0) / cv - 1.0;
                            const double X = x + s * (ct * u - st * v);
                            const double Y = y + s * (st * u + ct * v);
                            xmin = fmin(xmin, X); xmax = fmax(xmax, X);
                            ymin = fmin(ymin, Y); ymax = fmax(ymax, Y);
                        }
                        const double mg = 1e-3;
                        const double fx0 = fmax(ceil(xmin - mg), 0.0);
                        const double fx1 = fmin(floor(xmax + mg), D.W - 1.0);
                        const double fy0 = fmax(ceil(ymin - mg), 0.0);
                        const double fy1 = fmin(floor(ymax + mg), D.H - 1.0);
                        if (fx0 <= fx1 && fy0 <= fy1) {
                            rec.px0 = (int)fx0; rec.px1 = (int)fx1;
                            rec.py0 = (int)fy0; rec.py1 = (int)fy1;
                            tx0 = rec.px0 / TS; tx1 = rec.px1 / TS;
                            ty0 = rec.py0 / TS; ty1 = rec.py1 / TS;
                        }
                    }
                }
            }
            recs[g] = rec;
        }
        wr.aU = rec.aU; wr.bU = rec.bU; wr.eU = rec.eU; wr.aV = rec.aV; wr.bV = rec.bV;
        wr.eV = rec.eV; wr.Ulo = rec.Ulo; wr.Uhi = rec.Uhi; wr.Vlo = rec.Vlo; wr.Vhi = rec.Vhi;
        wr.tx0 = tx0; wr.tx1 = tx1; wr.ty0 = ty0; wr.ty1 = ty1;
        if (tx0 <= tx1) span = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
    }
    if (threadIdx.x < 64) {  // wave 0: scan of the spans (lanes past PREP_PRIMS add 0)
        int x = span;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if ((int)threadIdx.x >= o) x += y;
        }
        if (threadIdx.x < PREP_PRIMS) s_span[threadIdx.x] = x - span;
        if (threadIdx.x == PREP_PRIMS - 1) s_span[PREP_PRIMS] = x;
    }
    __syncthreads();
    // The (primitive, tile of its span) pairs of the workgroup's primitives are dealt over all
    // its threads, so a primitive spanning many tiles does not serialise its appends (returning
    // atomics) on a few lanes; each hit appends the primitive's row to the tile's list.
    const int total = s_span[PREP_PRIMS];
    for (int k = threadIdx.x; k < total; k += PREP_THREADS) {
        int pl = 0;  // the primitive whose span holds pair k: last pl with s_span[pl] <= k
#pragma unroll
        for (int step = PREP_PRIMS / 2; step > 0; step >>= 1)
            if (s_span[pl + step] <= k) pl += step;
        const WalkRec &r = s_rec[pl];
        const int g = (int)((long long)blockIdx.x * PREP_PRIMS + pl);
        const int kk = k - s_span[pl], nx = r.tx1 - r.tx0 + 1;
        const int tx = r.tx0 + kk % nx, ty = r.ty0 + kk / nx;
        const int X0 = tx * TS, X1 = min(X0 + TS - 1, r.W - 1);
        const int Y0 = ty * TS, Y1 = min(Y0 + TS - 1, r.H - 1);
        if (!tile_hits(r, X0, X1, Y0, Y1)) continue;
        const int tt = r.tile_off + ty * r.ntx + tx;
        const int pos = atomicAdd(&tile_count[tt], 1);
        if (pos < list_cap) {
            lists[(size_t)tt * list_cap + pos] = g;
        } else if (pos == list_cap) {  // the first entry that does not fit
            flags[F_S_OVERFLOW] = 1;
        }
    }
}

// ------------------------------------------------------------------------------------------
// Host launcher
// ------------------------------------------------------------------------------------------
hipError_t launch_binning(const BinArgs &a, hipStream_t st)
{
    if (a.pad_atlas) {
        if (a.dtype == 0)
            k_setup<float><<<a.B, SETUP_THREADS, 0, st>>>((const float *)a.atlas, a.B, a.Hb, a.Wb,
                                                           (float *)a.atlas_pad, a.Wp, a.box);
        else if (a.dtype == 2)
            k_setup<_Float16><<<a.B, SETUP_THREADS, 0, st>>>((const _Float16 *)a.atlas, a.B, a.Hb,
                                                              a.Wb, (_Float16 *)a.atlas_pad, a.Wp,
                                                              a.box);
        else
            k_setup<uint16_t><<<a.B, SETUP_THREADS, 0, st>>>((const uint16_t *)a.atlas, a.B, a.Hb,
                                                              a.Wb, (uint16_t *)a.atlas_pad, a.Wp,
                                                              a.box);
    }
    // small canvases: one extra binning workgroup orders the tiles by the previous forward's
    // list lengths, off the critical path; larger ones: the many-workgroup ordering of this
    // forward's lengths
    const bool order_in_prep = a.order && a.n_tiles <= ORDER_IN_PREP_MAX;
    auto prep = [&](auto kern, int pp) {
        const long long n_prep = (a.n_rows + pp - 1) / pp;
        const long long blocks = n_prep + (order_in_prep ? 1 : 0);
        if (blocks > 0)
            kern<<<(unsigned)blocks, PREP_THREADS, 0, st>>>(
                a.params, a.idx, a.n_rows, a.imgs, a.n_images, a.box, a.B, a.Hb, a.Wb, a.Wp,
                a.alpha_max, a.TS, a.recs, a.tile_count, a.lists, a.list_cap, a.flags,
                a.n_tiles, order_in_prep ? a.order : nullptr, a.prev_len, a.adam);
    };
    if (a.n_rows <= PREP_SMALL_N)
        prep(k_prep<16>, 16);
    else
        prep(k_prep<64>, 64);
    if (a.order && !order_in_prep && a.n_tiles > 0) {
        const int G = (a.n_tiles + ORDER_CHUNK - 1) / ORDER_CHUNK;
        k_order_count<<<G, ORDER_THREADS, 0, st>>>(a.tile_count, a.n_tiles, a.order_hist);
        k_order_scan<<<1, ORDER_BINS, 0, st>>>(a.order_hist, G);
        k_order_place<<<G, ORDER_THREADS, 0, st>>>(a.tile_count, a.n_tiles, a.order_hist,
                                                     a.order);
    }
    return hipGetLastError();
}

}  // namespace dbmp
