// dbmp_render_mse_noalloc: the fused render + MSE backward of dbmp_render_mse for callers that
// cannot allocate device memory. The workspace that a context would own (padded atlas, bitmap
// boxes, per-primitive records, tile counters and lists, per-pixel (K, T_K), per-tile losses,
// statistics) lives in one file-scope device array of fixed size instead; the kernels are the
// context path's own, given addresses inside that array.
//
// The array is resolved per device, once, by hipGetSymbolAddress: in host code its name is only
// a stand-in for the symbol, never a device address, so every launch uses the address kept for
// the device. Every call on a device shares that device's array, which keeps the last call's
// contents: the tile counters and the status words are cleared by a kernel at the start of each
// call (no hipMemsetAsync, so the call can be captured into a graph), and everything else is
// written before it is read within the call.
#include "dbmp_internal.h"
#include "diffbmp.h"
#include "workspace.h"

#include <limits.h>

#include <algorithm>
#include <mutex>

namespace dbmp {
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)DBMP_NOALLOC_SCRATCH_MB << 20;
}

static __device__ __align__(256) unsigned char scratch[dbmp::NOALLOC_SCRATCH_BYTES];

using namespace dbmp;

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_scratch[MAX_DEVICES] = {};
int g_ncu[MAX_DEVICES] = {};

// The device's address of `scratch` and its compute-unit count, resolved on the first call on
// that device (with it current).
int scratch_address(int dev, unsigned char **p, int *n_cu)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *q = nullptr;
        if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) {
            (void)hipGetLastError();
            return DBMP_EHIP;
        }
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            n < 1)
            n = 256;
        g_scratch[dev] = q;
        g_ncu[dev] = n;
    }
    *p = (unsigned char *)g_scratch[dev];
    *n_cu = g_ncu[dev];
    return DBMP_OK;
}

// Offsets of the call's buffers inside the scratch array (every region 256-byte aligned).
struct Layout {
    size_t desc, tile_count, tile_len, loss_tile, list_max, counter, box, atlas, recs, lists,
        saveK, saveT, total;
};

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout layout(long long N, int B, int Hb, int Wb, size_t esz, long long n_tiles, int cap,
              long long n_pix)
{
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += up256(bytes);
        return at;
    };
    L.desc = take(sizeof(ImgDev));
    L.tile_count = take(4 * (size_t)n_tiles);
    L.tile_len = take(4 * (size_t)n_tiles);
    L.loss_tile = take(4 * (size_t)n_tiles);
    L.list_max = take(4 * (size_t)DBMP_COUNTER_SLOTS);
    L.counter = take(8 * (size_t)DBMP_COUNTER_SLOTS);
    L.box = take(16 * (size_t)B);
    L.atlas = take(esz * (size_t)padded_atlas_elems(B, Hb, Wb));
    L.recs = take(sizeof(PrimRec) * (size_t)N);
    L.lists = take(4 * (size_t)n_tiles * (size_t)cap);
    L.saveK = take(4 * (size_t)n_pix);
    L.saveT = take(4 * (size_t)n_pix);
    L.total = o;
    return L;
}

// Start of a call: the image descriptor (passed by value) is written, and the tile counters and
// the caller's status words are cleared.
__global__ void k_noalloc_begin(ImgDev d, ImgDev *__restrict__ dst, int *__restrict__ tile_count,
                                int n_tiles, int *__restrict__ status)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *dst = d;
    if (i < 4) status[i] = 0;
    if (i < n_tiles) tile_count[i] = 0;
}

}  // namespace

extern "C" int dbmp_render_mse_noalloc(dbmp_stream stream, const float *params,
                                       const int32_t *atlas_idx, int N, const void *atlas, int B,
                                       int Hb, int Wb, int atlas_dtype, int H, int W,
                                       const float *bg, int bg_per_pixel, float alpha_max,
                                       int tile, int list_capacity, const float *target,
                                       float *image, float *dL_dparams, int accumulate,
                                       int32_t *status, size_t *scratch_bytes)
{
    // ---- host checks: nothing is enqueued and no HIP call is made before they pass ----
    if (N < 0 || H < 1 || W < 1 || (long long)H * W >= INT_MAX) return DBMP_EINVAL;
    if (!atlas || B < 1 || Hb < 2 || Wb < 2) return DBMP_EINVAL;
    if (atlas_dtype != DBMP_F32 && atlas_dtype != DBMP_BF16 && atlas_dtype != DBMP_F16)
        return DBMP_EINVAL;
    if (!bg || !target || !image || !status) return DBMP_EINVAL;
    if (N > 0 && (!params || !atlas_idx || !dL_dparams)) return DBMP_EINVAL;
    if (!(alpha_max > 0.f && alpha_max <= 1.f)) return DBMP_EINVAL;
    if (tile == 0) tile = DBMP_DEFAULT_TILE;
    if (tile != 8 && tile != 16 && tile != 32) return DBMP_EINVAL;
    if (list_capacity < 1 || list_capacity >= (1 << 24)) return DBMP_EINVAL;
    const size_t esz = atlas_dtype == DBMP_F32 ? 4 : 2;
    if (!atlas_addressable(B, Hb, Wb, (long long)esz)) return DBMP_EINVAL;
    const int cap = (list_capacity + 31) & ~31;
    const int ntx = (W + tile - 1) / tile, nty = (H + tile - 1) / tile;
    const long long n_tiles = (long long)ntx * nty;
    const Layout L = layout(N, B, Hb, Wb, esz, n_tiles, cap, (long long)H * W);
    if (scratch_bytes) *scratch_bytes = L.total;
    if (L.total > NOALLOC_SCRATCH_BYTES) return DBMP_ENOMEM;  // beyond the fixed scratch

    // ---- the device's scratch array ----
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return DBMP_EHIP;
    unsigned char *S = nullptr;
    int n_cu = 256;
    int rc = scratch_address(dev, &S, &n_cu);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;

    ImgDev D{};
    D.H = H; D.W = W; D.N = N; D.ntx = ntx; D.nty = nty; D.tile_off = 0;
    D.prim_off = 0; D.pix_off = 0;
    ImgDev *d_img = (ImgDev *)(S + L.desc);
    int *tile_count = (int *)(S + L.tile_count);
    const int nb = (int)((std::max(n_tiles, 4LL) + 255) / 256);
    k_noalloc_begin<<<nb, 256, 0, st>>>(D, d_img, tile_count, (int)n_tiles, status);

    // padding of the atlas, then per-primitive setup and binning (the context path's kernels)
    BinArgs ba{};
    ba.params = params; ba.idx = atlas_idx; ba.n_rows = N;
    ba.imgs = d_img; ba.n_images = 1; ba.n_tiles = (int)n_tiles;
    ba.atlas = atlas; ba.dtype = atlas_dtype; ba.B = B; ba.Hb = Hb; ba.Wb = Wb; ba.Wp = Wb + 2;
    ba.alpha_max = alpha_max; ba.TS = tile;
    ba.atlas_pad = S + L.atlas; ba.box = (int *)(S + L.box);
    ba.recs = (PrimRec *)(S + L.recs);
    ba.tile_count = tile_count; ba.lists = (int *)(S + L.lists); ba.list_cap = cap;
    ba.flags = status;  // the status words are the flag slots {overflow, bad index, non-finite}
    ba.pad_atlas = true;
    ba.order = nullptr; ba.order_hist = nullptr; ba.prev_len = nullptr;
    hipError_t e = launch_binning(ba, st);
    if (e != hipSuccess) return DBMP_EHIP;
    if (!accumulate && N > 0) {
        e = launch_fill0(dL_dparams, (long long)N * 8, st);
        if (e != hipSuccess) return DBMP_EHIP;
    }

    RasterArgs ra{};
    ra.recs = (const PrimRec *)(S + L.recs);
    ra.lists = (const int *)(S + L.lists);
    ra.list_cap = cap;
    ra.tile_count = tile_count;
    ra.tile_len = (int *)(S + L.tile_len);
    ra.list_max = (int *)(S + L.list_max);
    ra.imgs = d_img;
    ra.n_images = 1; ra.n_tiles = (int)n_tiles;
    ra.atlas_pad = S + L.atlas; ra.dtype = atlas_dtype; ra.Wp = Wb + 2; ra.Hb = Hb; ra.Wb = Wb;
    ra.zcell = (int)zero_cell(B, Hb, Wb);
    ra.bg = bg; ra.bg_pp = bg_per_pixel ? 1 : 0; ra.image = image; ra.alpha = nullptr;
    ra.saveK = (int *)(S + L.saveK); ra.saveT = (float *)(S + L.saveT);
    ra.flags = status; ra.TS = tile;
    ra.pair_counter = (unsigned long long *)(S + L.counter);
    ra.loss_tile = (float *)(S + L.loss_tile);
    ra.sched = SCHED_GRID; ra.grid = 0; ra.grab = 0; ra.n_cu = n_cu;
    ra.order = nullptr; ra.queue = nullptr;
    ra.target = target; ra.dparams = dL_dparams;
    ra.fit_state = nullptr;
    e = launch_raster_fwd(ra, st);
    return e == hipSuccess ? DBMP_OK : DBMP_EHIP;
}
