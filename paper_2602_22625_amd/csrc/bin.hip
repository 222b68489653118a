// Per-primitive setup and screen-tile binning (Sec. 3.1.1 "Parallelization": each primitive is
// assigned to every T x T tile its footprint overlaps; lists are composited front to back).
//
// Stages, all on the device and all asynchronous:
//   k_setup    pads every bitmap with a one-texel zero border (the zero padding of the bilinear
//              sampler), finds each bitmap's tight non-zero box, clears counters and flags;
//   k_prep     per primitive: sigmoid/exp/sincos, the inverse affine map of Eqs. (1)-(2) folded
//              into U' = aU x + bU y + eU (float64), the exact support parallelogram, its tile
//              span, and a count per overlapped tile (separating-axis test, so rotated
//              primitives are not charged for the corners of their bounding box);
//   k_scan     exclusive scan of the per-tile counts -> per-tile list starts, overflow check;
//   k_emit     writes primitive ids into their tiles' lists (order within a tile arbitrary);
//   k_sort     sorts every tile's list ascending = front to back (depth order = index order).
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
        int *__restrict__ box, int *__restrict__ tile_count, int n_tiles, int *__restrict__ flags)
{
    const int Hp = Hb + 2;
    if ((int)blockIdx.x < B) {
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
    } else {
        const int nb = gridDim.x - B, ib = blockIdx.x - B;
        for (int i = ib * blockDim.x + threadIdx.x; i < n_tiles; i += nb * blockDim.x)
            tile_count[(size_t)i * CNT_STRIDE] = 0;
        if (ib == 0 && threadIdx.x < F_S_OVERFLOW) flags[threadIdx.x] = 0;  // per-forward flags
    }
}

// ------------------------------------------------------------------------------------------
// Separating-axis test of the support parallelogram against a tile's pixel centres. U' and V'
// are affine in (x, y), so their range over the tile rectangle is attained at its corners; the
// tile's own axes are covered by the bounding-box span. The margin keeps the test conservative
// against rounding; the raster kernels test every pixel exactly.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ bool tile_hits(const PrimRec &r, int X0, int X1, int Y0, int Y1)
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
// k_prep: one thread per (global) primitive row.
// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_prep(const float *__restrict__ params, const int *__restrict__ idx, long long n_rows,
       const ImgDev *__restrict__ imgs, int n_images, const int *__restrict__ box, int B, int Hb,
       int Wb, int Wp, float alpha_max, int TS, PrimRec *__restrict__ recs,
       int *__restrict__ tile_count, int *__restrict__ flags)
{
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_rows) return;
    PrimRec rec;
    rec.aU = rec.bU = rec.eU = rec.aV = rec.bV = rec.eV = 0.0;
    rec.Ulo = 1.0; rec.Uhi = 0.0; rec.Vlo = 1.0; rec.Vhi = 0.0;  // empty support
    rec.ka = 0.f; rec.cr = rec.cg = rec.cb = 0.f; rec.tex = 0; rec.omsig = 1.f;
    rec.faU = rec.fbU = rec.faV = rec.fbV = 0.f;
    rec.tx0 = 1; rec.tx1 = 0; rec.ty0 = 1; rec.ty1 = 0;
    rec.pad[0] = rec.pad[1] = rec.pad[2] = 0;
    const int b = find_by_prim(imgs, n_images, g);
    const ImgDev D = imgs[b];
    rec.img = b;
    const bool in_image = g >= D.prim_off && g < D.prim_off + D.N;
    if (in_image) {
        float p[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) p[j] = params[g * 8 + j];
        const int k = idx[g];
        bool ok = true;
        if (k < 0 || k >= B) {
            atomicOr(&flags[F_BADIDX], 1);
            atomicOr(&flags[F_S_BADIDX], 1);
            ok = false;
        }
        bool fin = true;
#pragma unroll
        for (int j = 0; j < 8; ++j) fin = fin && isfinite(p[j]);
        const double s = exp((double)p[2]);
        if (!(s > 0.0) || !isfinite(s)) fin = false;  // scale underflows or overflows
        if (!fin) {
            atomicOr(&flags[F_NONFINITE], 1);
            atomicOr(&flags[F_S_NONFINITE], 1);
            ok = false;
        }
        if (ok) {
            double st, ct;
            sincos((double)p[3], &st, &ct);
            const double inv_s = 1.0 / s;
            const double cu = 0.5 * (Wb - 1), cv = 0.5 * (Hb - 1);  // dU/du, dV/dv of Eq. (2)
            const double x = p[0], y = p[1];
            // Eq. (1)-(2): u = (ct dx + st dy)/s, v = (-st dx + ct dy)/s, U = cu (u + 1), plus the
            // one-texel shift into the padded bitmap.
            rec.aU = cu * ct * inv_s;  rec.bU = cu * st * inv_s;
            rec.aV = -cv * st * inv_s; rec.bV = cv * ct * inv_s;
            rec.eU = (cu + 1.0) - rec.aU * x - rec.bU * y;
            rec.eV = (cv + 1.0) - rec.aV * x - rec.bV * y;
            rec.faU = (float)rec.aU; rec.fbU = (float)rec.bU;
            rec.faV = (float)rec.aV; rec.fbV = (float)rec.bV;
            const double sig = 1.0 / (1.0 + exp(-(double)p[4]));
            rec.ka = (float)(alpha_max * sig);
            rec.omsig = (float)(1.0 / (1.0 + exp((double)p[4])));  // 1 - sigmoid, no cancellation
            rec.cr = (float)(1.0 / (1.0 + exp(-(double)p[5])));
            rec.cg = (float)(1.0 / (1.0 + exp(-(double)p[6])));
            rec.cb = (float)(1.0 / (1.0 + exp(-(double)p[7])));
            const int Hp = Hb + 2;
            rec.tex = k * Hp * Wp;
            int xlo = box[4 * k];
            const int xhi = box[4 * k + 1];
            const int ylo = box[4 * k + 2], yhi = box[4 * k + 3];
            if (xlo == INT_MIN) {  // the bitmap holds a non-finite texel (read as 0)
                atomicOr(&flags[F_NONFINITE], 1);
                atomicOr(&flags[F_S_NONFINITE], 1);
                xlo = 0;
            }
            if (xlo <= xhi && D.W > 0 && D.H > 0) {
                // floor(U') in [xlo, xhi + 1] reads at least one non-zero texel (padded columns
                // xlo + 1 .. xhi + 1); elsewhere M and its derivatives are exactly zero.
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
                const double fx0 = fmax(ceil(xmin - mg), 0.0), fx1 = fmin(floor(xmax + mg), D.W - 1.0);
                const double fy0 = fmax(ceil(ymin - mg), 0.0), fy1 = fmin(floor(ymax + mg), D.H - 1.0);
                if (fx0 <= fx1 && fy0 <= fy1) {
                    rec.tx0 = (int)fx0 / TS; rec.tx1 = (int)fx1 / TS;
                    rec.ty0 = (int)fy0 / TS; rec.ty1 = (int)fy1 / TS;
                }
            }
        }
    }
    recs[g] = rec;
}

// k_count: 16 lanes per primitive walk its tile span and count the tiles its support hits.
__global__ void __launch_bounds__(256)
k_count(const PrimRec *__restrict__ recs, long long n_rows, const ImgDev *__restrict__ imgs,
        int TS, int *__restrict__ tile_count)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long g = t / 16;
    const int l = (int)(t % 16);
    if (g >= n_rows) return;
    const PrimRec &r = recs[g];
    if (r.tx0 > r.tx1) return;
    const ImgDev D = imgs[r.img];
    const int nx = r.tx1 - r.tx0 + 1, ny = r.ty1 - r.ty0 + 1;
    for (int k = l; k < nx * ny; k += 16) {
        const int tx = r.tx0 + k % nx, ty = r.ty0 + k / nx;
        const int X0 = tx * TS, X1 = min(X0 + TS - 1, D.W - 1);
        const int Y0 = ty * TS, Y1 = min(Y0 + TS - 1, D.H - 1);
        if (tile_hits(r, X0, X1, Y0, Y1))
            atomicAdd(&tile_count[(size_t)(D.tile_off + ty * D.ntx + tx) * CNT_STRIDE], 1);
    }
}

// ------------------------------------------------------------------------------------------
// k_scan: one workgroup of 1024 threads; exclusive scan of tile_count into tile_start, then
// tile_count is zeroed to serve as the fill counter of k_emit (which restores it).
// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(1024)
k_scan(int *__restrict__ tile_count, int *__restrict__ tile_start, int n_tiles,
       long long pair_cap, int *__restrict__ flags)
{
    constexpr int PER = 4;
    __shared__ long long wsum[16];
    __shared__ long long carry_s;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (t == 0) carry_s = 0;
    __syncthreads();
    for (int base = 0; base < n_tiles; base += 1024 * PER) {
        int v[PER];
        long long loc = 0;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int j = base + t * PER + i;
            v[i] = j < n_tiles ? tile_count[(size_t)j * CNT_STRIDE] : 0;
            loc += v[i];
        }
        // inclusive wave scan of loc
        long long inc = loc;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const long long o = __shfl_up(inc, d);
            if (lane >= d) inc += o;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        long long wpre = 0;
        for (int i = 0; i < w; ++i) wpre += wsum[i];
        long long run = carry_s + wpre + inc - loc;  // exclusive prefix of this thread
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int j = base + t * PER + i;
            if (j < n_tiles) {
                tile_start[j] = (int)(run < INT_MAX ? run : INT_MAX);
                tile_count[(size_t)j * CNT_STRIDE] = 0;
            }
            run += v[i];
        }
        __syncthreads();
        if (t == 1023) carry_s = run;
        __syncthreads();
    }
    if (t == 0) {
        const long long total = carry_s;
        const int tc = (int)(total < INT_MAX ? total : INT_MAX);
        flags[F_TOTAL] = tc;
        atomicMax(&flags[F_S_TOTALMAX], tc);
        if (total > pair_cap) {
            flags[F_OVERFLOW] = 1;
            flags[F_S_OVERFLOW] = 1;
        }
    }
}

// ------------------------------------------------------------------------------------------
// k_emit: appends each primitive's row to the lists of the tiles it hits. Sixteen lanes share
// a primitive and split its tile span, so its (returning) atomics are issued together instead
// of one after another.
// ------------------------------------------------------------------------------------------
#define EMIT_LANES 16

__global__ void __launch_bounds__(256)
k_emit(const PrimRec *__restrict__ recs, long long n_rows, const ImgDev *__restrict__ imgs, int TS,
       const int *__restrict__ tile_start, int *__restrict__ tile_fill, int *__restrict__ pairs,
       long long pair_cap)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long g = t / EMIT_LANES;
    const int l = (int)(t % EMIT_LANES);
    if (g >= n_rows) return;
    const PrimRec &r = recs[g];
    if (r.tx0 > r.tx1) return;
    const ImgDev D = imgs[r.img];
    const int nx = r.tx1 - r.tx0 + 1, ny = r.ty1 - r.ty0 + 1;
    for (int k = l; k < nx * ny; k += EMIT_LANES) {
        const int tx = r.tx0 + k % nx, ty = r.ty0 + k / nx;
        const int X0 = tx * TS, X1 = min(X0 + TS - 1, D.W - 1);
        const int Y0 = ty * TS, Y1 = min(Y0 + TS - 1, D.H - 1);
        if (!tile_hits(r, X0, X1, Y0, Y1)) continue;
        const int tt = D.tile_off + ty * D.ntx + tx;
        const long long pos =
            (long long)tile_start[tt] + atomicAdd(&tile_fill[(size_t)tt * CNT_STRIDE], 1);
        if (pos < pair_cap) pairs[pos] = (int)g;
    }
}

// ------------------------------------------------------------------------------------------
// k_sort: one wave per tile, ascending order (front to back). Lists of up to 64 entries are
// ranked in registers; up to SORT_LDS entries are sorted in LDS; longer lists in place in global
// memory. The bitonic network uses only ascending comparators (the first sub-stage of every
// merge compares i with i ^ (k - 1)), so a list of any length n behaves as if padded with +inf
// and comparators reaching past n are skipped.
// ------------------------------------------------------------------------------------------
#define SORT_LDS 2048

template <typename Buf>
__device__ __forceinline__ void bitonic_asc(Buf &a, int n, int lane)
{
    int N2 = 1;
    while (N2 < n) N2 <<= 1;
    for (int k = 2; k <= N2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < N2; i += 64) {
                const int l = (j == (k >> 1)) ? (i ^ (k - 1)) : (i ^ j);
                if (l > i && l < n) {
                    const int x = a.get(i), y = a.get(l);
                    if (y < x) { a.set(i, y); a.set(l, x); }
                }
            }
            a.sync();
        }
    }
}

struct LdsBuf {
    int *p;
    __device__ int get(int i) const { return p[i]; }
    __device__ void set(int i, int v) { p[i] = v; }
    __device__ void sync() { __syncthreads(); }
};
struct GlobalBuf {  // one wave on one CU: volatile loads read through to L2
    int *p;
    __device__ int get(int i) const { return ((volatile int *)p)[i]; }
    __device__ void set(int i, int v) { ((volatile int *)p)[i] = v; }
    __device__ void sync() { __threadfence_block(); __syncthreads(); }
};

__global__ void __launch_bounds__(64)
k_sort(int *__restrict__ pairs, const int *__restrict__ tile_start,
       const int *__restrict__ tile_count, int n_tiles, const int *__restrict__ flags)
{
    if (flags[F_OVERFLOW]) return;
    const int t = blockIdx.x;
    if (t >= n_tiles) return;
    const int lane = threadIdx.x;
    const int n = tile_count[(size_t)t * CNT_STRIDE];
    if (n <= 1) return;
    int *seg = pairs + tile_start[t];
    if (n <= 64) {
        const int v = lane < n ? seg[lane] : INT_MAX;
        int rank = 0;
        for (int k = 0; k < n; ++k) rank += (__shfl(v, k) < v);
        if (lane < n) seg[rank] = v;
        return;
    }
    if (n <= SORT_LDS) {
        __shared__ int buf[SORT_LDS];
        for (int i = lane; i < n; i += 64) buf[i] = seg[i];
        __syncthreads();
        LdsBuf b{buf};
        bitonic_asc(b, n, lane);
        for (int i = lane; i < n; i += 64) seg[i] = buf[i];
        return;
    }
    GlobalBuf gb{seg};
    bitonic_asc(gb, n, lane);
}

// ------------------------------------------------------------------------------------------
// Host launchers
// ------------------------------------------------------------------------------------------

hipError_t launch_binning(const BinArgs &a, hipStream_t st)
{
    const int zb = a.n_tiles > 0 ? min((a.n_tiles + SETUP_THREADS - 1) / SETUP_THREADS, 256) : 1;
    if (a.dtype == 0)
        k_setup<float><<<a.B + zb, SETUP_THREADS, 0, st>>>((const float *)a.atlas, a.B, a.Hb, a.Wb,
                                                  (float *)a.atlas_pad, a.Wp, a.box, a.tile_count,
                                                  a.n_tiles, a.flags);
    else
        k_setup<uint16_t><<<a.B + zb, SETUP_THREADS, 0, st>>>((const uint16_t *)a.atlas, a.B, a.Hb, a.Wb,
                                                     (uint16_t *)a.atlas_pad, a.Wp, a.box,
                                                     a.tile_count, a.n_tiles, a.flags);
    if (a.n_rows > 0)
        k_prep<<<(unsigned)((a.n_rows + 255) / 256), 256, 0, st>>>(
            a.params, a.idx, a.n_rows, a.imgs, a.n_images, a.box, a.B, a.Hb, a.Wb, a.Wp,
            a.alpha_max, a.TS, a.recs, a.tile_count, a.flags);
    if (a.n_rows > 0)
        k_count<<<(unsigned)((a.n_rows * 16 + 255) / 256), 256, 0, st>>>(a.recs, a.n_rows, a.imgs,
                                                                          a.TS, a.tile_count);
    k_scan<<<1, 1024, 0, st>>>(a.tile_count, a.tile_start, a.n_tiles, a.pair_cap, a.flags);
    if (a.n_rows > 0)
        k_emit<<<(unsigned)((a.n_rows * EMIT_LANES + 255) / 256), 256, 0, st>>>(
            a.recs, a.n_rows, a.imgs, a.TS, a.tile_start, a.tile_count, a.pairs, a.pair_cap);
    if (a.n_tiles > 0)
        k_sort<<<a.n_tiles, 64, 0, st>>>(a.pairs, a.tile_start, a.tile_count, a.n_tiles, a.flags);
    return hipGetLastError();
}

}  // namespace dbmp
