// C ABI of the rasteriser (declared in include/diffbmp.h): context, workspace and launches.
#include "dbmp_internal.h"
#include "diffbmp.h"

#include <limits.h>
#include <stdio.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>


using namespace dbmp;

namespace {

struct Buf {
    void *p = nullptr;
    size_t cap = 0;  // bytes
};

}  // namespace

struct dbmp_ctx {
    int device = 0;
    std::string err;
    Buf recs, tile_count, tile_start, pairs, saveK, saveT, atlas_pad, box, imgs, flags, counter;
    long long pair_cap = 0;
    std::vector<ImgDev> imgs_uploaded;  // what the device copy of the descriptors holds
    // state of the last forward, for the backward
    bool have_fwd = false;
    RasterArgs ra{};
    long long n_rows = 0;
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int fail(dbmp_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

int hip_fail(dbmp_ctx *c, hipError_t e, const char *what)
{
    return fail(c, DBMP_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool capturing(hipStream_t st)
{
    hipStreamCaptureStatus s = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &s) != hipSuccess) return false;
    return s != hipStreamCaptureStatusNone;
}

// Grows `b` to at least `bytes` (contents not preserved). Synchronous; refused while the stream
// is being captured into a graph.
int ensure(dbmp_ctx *c, Buf &b, size_t bytes, hipStream_t st, const char *what)
{
    if (bytes == 0) bytes = 16;
    if (b.cap >= bytes) return DBMP_OK;
    if (capturing(st))
        return fail(c, DBMP_ESTATE, std::string("workspace '") + what +
                                        "' must grow during graph capture; run the call once "
                                        "before capturing");
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
    const size_t want = bytes + bytes / 4;
    e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return fail(c, DBMP_ENOMEM, std::string("hipMalloc failed for ") + what);
    }
    b.cap = want;
    return DBMP_OK;
}

bool same_imgs(const std::vector<ImgDev> &a, const std::vector<ImgDev> &b)
{
    if (a.size() != b.size()) return false;
    for (size_t i = 0; i < a.size(); ++i)
        if (a[i].H != b[i].H || a[i].W != b[i].W || a[i].N != b[i].N ||
            a[i].ntx != b[i].ntx || a[i].nty != b[i].nty || a[i].tile_off != b[i].tile_off ||
            a[i].prim_off != b[i].prim_off || a[i].pix_off != b[i].pix_off)
            return false;
    return true;
}

// Shared body of dbmp_render and dbmp_render_batched.
int render_impl(dbmp_ctx *c, hipStream_t st, const std::vector<dbmp_image_desc> &descs,
                const float *params, const int32_t *atlas_idx, const void *atlas, int B, int Hb,
                int Wb, int dtype, const float *bg, int bg_pp, float alpha_max, int tile,
                float *image, float *alpha)
{
    if (!atlas || B < 1 || Hb < 2 || Wb < 2) return fail(c, DBMP_EINVAL, "bad atlas shape");
    if (dtype != DBMP_F32 && dtype != DBMP_BF16) return fail(c, DBMP_EINVAL, "bad atlas dtype");
    if (!bg) return fail(c, DBMP_EINVAL, "bg is NULL");
    if (!(alpha_max > 0.f && alpha_max <= 1.f))
        return fail(c, DBMP_EINVAL, "alpha_max must be in (0, 1]");
    if (tile != 8 && tile != 16 && tile != 32)
        return fail(c, DBMP_EINVAL, "tile must be 8, 16 or 32");
    if (!image) return fail(c, DBMP_EINVAL, "image is NULL");
    const int Hp = Hb + 2, Wp = Wb + 2;
    if ((long long)B * Hp * Wp >= INT_MAX) return fail(c, DBMP_EINVAL, "atlas too large");

    std::vector<ImgDev> imgs(descs.size());
    long long n_rows = 0, tiles = 0, n_pix = 0, prev_end = 0;
    for (size_t i = 0; i < descs.size(); ++i) {
        const dbmp_image_desc &d = descs[i];
        if (d.H < 1 || d.W < 1 || d.N < 0 || d.prim_offset < 0 || d.pixel_offset < 0)
            return fail(c, DBMP_EINVAL, "bad image descriptor " + std::to_string(i));
        if ((long long)d.H * d.W >= INT_MAX)
            return fail(c, DBMP_EINVAL, "image too large " + std::to_string(i));
        if (d.prim_offset < prev_end)
            return fail(c, DBMP_EINVAL,
                        "descriptors must have increasing, non-overlapping primitive ranges");
        prev_end = d.prim_offset + d.N;
        ImgDev &g = imgs[i];
        g.H = d.H; g.W = d.W; g.N = d.N;
        g.ntx = (d.W + tile - 1) / tile;
        g.nty = (d.H + tile - 1) / tile;
        g.tile_off = (int)tiles;
        g.pad0 = g.pad1 = 0;
        g.prim_off = d.prim_offset;
        g.pix_off = d.pixel_offset;
        tiles += (long long)g.ntx * g.nty;
        n_rows = prev_end;
        n_pix = std::max(n_pix, (long long)d.pixel_offset + (long long)d.H * d.W);
        if (tiles >= INT_MAX) return fail(c, DBMP_EINVAL, "too many tiles");
    }
    if (n_rows > 0 && (!params || !atlas_idx))
        return fail(c, DBMP_EINVAL, "params / atlas_idx is NULL");
    if (n_rows >= INT_MAX) return fail(c, DBMP_EINVAL, "too many primitives");

    int rc;
    const size_t ni = imgs.size();
    if ((rc = ensure(c, c->recs, sizeof(PrimRec) * (size_t)n_rows, st, "records"))) return rc;
    if ((rc = ensure(c, c->tile_count, 4 * CNT_STRIDE * (size_t)tiles, st, "tile_count")))
        return rc;
    if ((rc = ensure(c, c->tile_start, 4 * (size_t)tiles, st, "tile_start"))) return rc;
    if ((rc = ensure(c, c->pairs, 4 * (size_t)c->pair_cap, st, "pairs"))) return rc;
    if ((rc = ensure(c, c->saveK, 4 * (size_t)n_pix, st, "saveK"))) return rc;
    if ((rc = ensure(c, c->saveT, 4 * (size_t)n_pix, st, "saveT"))) return rc;
    const size_t esz = dtype == DBMP_F32 ? 4 : 2;
    if ((rc = ensure(c, c->atlas_pad, esz * (size_t)B * Hp * Wp, st, "atlas"))) return rc;
    if ((rc = ensure(c, c->box, 16 * (size_t)B, st, "boxes"))) return rc;
    if ((rc = ensure(c, c->flags, 4 * F_COUNT, st, "flags"))) return rc;
    if (c->imgs.cap < sizeof(ImgDev) * ni || !same_imgs(imgs, c->imgs_uploaded)) {
        if (capturing(st))
            return fail(c, DBMP_ESTATE,
                        "image descriptors changed during graph capture; run the call once "
                        "before capturing");
        if ((rc = ensure(c, c->imgs, sizeof(ImgDev) * ni, st, "descriptors"))) return rc;
        hipError_t e = hipStreamSynchronize(st);  // earlier launches may still read the table
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
        e = hipMemcpy(c->imgs.p, imgs.data(), sizeof(ImgDev) * ni, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(c, e, "descriptor upload");
        c->imgs_uploaded = imgs;
    }

    BinArgs ba{};
    ba.params = params; ba.idx = atlas_idx; ba.n_rows = n_rows;
    ba.imgs = (const ImgDev *)c->imgs.p; ba.n_images = (int)ni; ba.n_tiles = (int)tiles;
    ba.atlas = atlas; ba.dtype = dtype; ba.B = B; ba.Hb = Hb; ba.Wb = Wb; ba.Wp = Wp;
    ba.alpha_max = alpha_max; ba.TS = tile; ba.atlas_pad = c->atlas_pad.p;
    ba.box = (int *)c->box.p; ba.recs = (PrimRec *)c->recs.p;
    ba.tile_count = (int *)c->tile_count.p; ba.tile_start = (int *)c->tile_start.p;
    ba.pairs = (int *)c->pairs.p; ba.pair_cap = c->pair_cap; ba.flags = (int *)c->flags.p;
    hipError_t e = launch_binning(ba, st);
    if (e != hipSuccess) return hip_fail(c, e, "binning launch");

    RasterArgs &ra = c->ra;
    ra = RasterArgs{};
    ra.recs = (const PrimRec *)c->recs.p;
    ra.pairs = (const int *)c->pairs.p;
    ra.tile_start = (const int *)c->tile_start.p;
    ra.tile_count = (const int *)c->tile_count.p;
    ra.imgs = (const ImgDev *)c->imgs.p;
    ra.n_images = (int)ni; ra.n_tiles = (int)tiles;
    ra.atlas_pad = c->atlas_pad.p; ra.dtype = dtype; ra.Wp = Wp; ra.Hb = Hb; ra.Wb = Wb;
    ra.bg = bg; ra.bg_pp = bg_pp; ra.image = image; ra.alpha = alpha;
    ra.saveK = (int *)c->saveK.p; ra.saveT = (float *)c->saveT.p;
    ra.flags = (const int *)c->flags.p; ra.TS = tile;
    ra.pair_counter = (unsigned long long *)c->counter.p;
    e = launch_raster_fwd(ra, st);
    if (e != hipSuccess) return hip_fail(c, e, "forward launch");
    c->have_fwd = true;
    c->n_rows = n_rows;
    c->err.clear();
    return DBMP_OK;
}

}  // namespace

extern "C" {

int dbmp_create(dbmp_ctx **out, int device, long long pair_capacity)
{
    if (!out || pair_capacity < 0 || pair_capacity >= INT_MAX) return DBMP_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return DBMP_EINVAL;
    dbmp_ctx *c = new (std::nothrow) dbmp_ctx();
    if (!c) return DBMP_ENOMEM;
    c->device = device;
    c->pair_cap = pair_capacity > 0 ? pair_capacity : (1LL << 20);
    DeviceGuard g(device);
    int rc = ensure(c, c->flags, 4 * F_COUNT, nullptr, "flags");
    if (rc) { delete c; return rc; }
    (void)hipMemset(c->flags.p, 0, 4 * F_COUNT);
    rc = ensure(c, c->counter, 8 * DBMP_COUNTER_SLOTS, nullptr, "counter");
    if (rc) { delete c; return rc; }
    (void)hipMemset(c->counter.p, 0, 8 * DBMP_COUNTER_SLOTS);
    (void)hipDeviceSynchronize();
    rc = ensure(c, c->pairs, 4 * (size_t)c->pair_cap, nullptr, "pairs");
    if (rc) { delete c; return rc; }
    c->pair_cap = (long long)(c->pairs.cap / 4);
    *out = c;
    return DBMP_OK;
}

int dbmp_destroy(dbmp_ctx *c)
{
    if (!c) return DBMP_EINVAL;
    {
        DeviceGuard g(c->device);
        (void)hipDeviceSynchronize();
        Buf *bs[] = {&c->recs, &c->tile_count, &c->tile_start, &c->pairs, &c->saveK,
                     &c->saveT, &c->atlas_pad, &c->box, &c->imgs, &c->flags, &c->counter};
        for (Buf *b : bs)
            if (b->p) (void)hipFree(b->p);
    }
    delete c;
    return DBMP_OK;
}

int dbmp_reserve(dbmp_ctx *c, long long pair_capacity)
{
    if (!c || pair_capacity < 0 || pair_capacity >= INT_MAX) return DBMP_EINVAL;
    if (pair_capacity <= c->pair_cap) return DBMP_OK;
    DeviceGuard g(c->device);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
    int rc = ensure(c, c->pairs, 4 * (size_t)pair_capacity, nullptr, "pairs");
    if (rc) return rc;
    c->pair_cap = std::min<long long>((long long)(c->pairs.cap / 4), INT_MAX - 1);
    e = hipMemset((int *)c->flags.p + F_S_TOTALMAX, 0, sizeof(int));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(c, e, "flag reset");
    c->have_fwd = false;  // the lists of the last forward are gone
    return DBMP_OK;
}

int dbmp_render(dbmp_ctx *c, dbmp_stream stream, const float *params, const int32_t *atlas_idx,
                int N, const void *atlas, int B, int Hb, int Wb, int atlas_dtype, int H, int W,
                const float *bg, int bg_per_pixel, float alpha_max, int tile, float *image,
                float *alpha)
{
    if (!c) return DBMP_EINVAL;
    if (N < 0 || H < 1 || W < 1) return fail(c, DBMP_EINVAL, "bad N / H / W");
    DeviceGuard g(c->device);
    std::vector<dbmp_image_desc> d(1);
    d[0].H = H; d[0].W = W; d[0].N = N; d[0].reserved = 0;
    d[0].prim_offset = 0; d[0].pixel_offset = 0;
    return render_impl(c, (hipStream_t)stream, d, params, atlas_idx, atlas, B, Hb, Wb,
                       atlas_dtype, bg, bg_per_pixel ? 1 : 0, alpha_max, tile, image, alpha);
}

int dbmp_render_batched(dbmp_ctx *c, dbmp_stream stream, int n_images,
                        const dbmp_image_desc *descs, const float *params,
                        const int32_t *atlas_idx, const void *atlas, int B, int Hb, int Wb,
                        int atlas_dtype, const float *bg, float alpha_max, int tile,
                        float *image, float *alpha)
{
    if (!c) return DBMP_EINVAL;
    if (n_images < 1 || !descs) return fail(c, DBMP_EINVAL, "need n_images >= 1 descriptors");
    DeviceGuard g(c->device);
    std::vector<dbmp_image_desc> d(descs, descs + n_images);
    return render_impl(c, (hipStream_t)stream, d, params, atlas_idx, atlas, B, Hb, Wb,
                       atlas_dtype, bg, 0, alpha_max, tile, image, alpha);
}

int dbmp_render_backward(dbmp_ctx *c, dbmp_stream stream, const float *dL_dimage,
                         const float *dL_dalpha, float *dL_dparams)
{
    if (!c) return DBMP_EINVAL;
    if (!c->have_fwd) return fail(c, DBMP_ESTATE, "no forward on this context");
    if (!dL_dimage || (c->n_rows > 0 && !dL_dparams))
        return fail(c, DBMP_EINVAL, "dL_dimage / dL_dparams is NULL");
    DeviceGuard g(c->device);
    RasterArgs a = c->ra;
    a.gI = dL_dimage;
    a.gA = dL_dalpha;
    a.dparams = dL_dparams;
    a.n_param_floats = c->n_rows * 8;
    hipError_t e = launch_raster_bwd(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "backward launch");
    c->err.clear();
    return DBMP_OK;
}

int dbmp_check(dbmp_ctx *c, dbmp_stream stream)
{
    if (!c) return DBMP_EINVAL;
    DeviceGuard g(c->device);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
    int f[F_COUNT];
    e = hipMemcpy(f, c->flags.p, sizeof(f), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "flag readback");
    if (f[F_S_OVERFLOW] | f[F_S_BADIDX] | f[F_S_NONFINITE]) {
        e = hipMemset((int *)c->flags.p + F_S_OVERFLOW, 0, 3 * sizeof(int));
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(c, e, "flag reset");
    }
    if (f[F_S_OVERFLOW])
        return fail(c, DBMP_EOVERFLOW, "pair buffer too small: " +
                                           std::to_string(f[F_S_TOTALMAX]) +
                                           " pairs needed, capacity " +
                                           std::to_string(c->pair_cap));
    if (f[F_S_BADIDX]) return fail(c, DBMP_EINVAL, "atlas index out of range");
    if (f[F_S_NONFINITE]) return fail(c, DBMP_ENONFINITE, "non-finite parameter or texel");
    return DBMP_OK;
}

long long dbmp_pair_count(dbmp_ctx *c, dbmp_stream stream)
{
    if (!c) return -1;
    DeviceGuard g(c->device);
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return -1;
    int f[F_COUNT];
    if (hipMemcpy(f, c->flags.p, sizeof(f), hipMemcpyDeviceToHost) != hipSuccess) return -1;
    return f[F_S_TOTALMAX];
}

long long dbmp_support_pairs(dbmp_ctx *c, dbmp_stream stream, int reset)
{
    if (!c) return -1;
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    if (hipStreamSynchronize(st) != hipSuccess) return -1;
    std::vector<unsigned long long> slots(DBMP_COUNTER_SLOTS);
    if (hipMemcpy(slots.data(), c->counter.p, 8 * DBMP_COUNTER_SLOTS, hipMemcpyDeviceToHost) !=
        hipSuccess)
        return -1;
    unsigned long long v = 0;
    for (unsigned long long x : slots) v += x;
    if (reset && hipMemset(c->counter.p, 0, 8 * DBMP_COUNTER_SLOTS) != hipSuccess) return -1;
    if (reset && hipDeviceSynchronize() != hipSuccess) return -1;
    return (long long)v;
}

const char *dbmp_last_error(const dbmp_ctx *c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
