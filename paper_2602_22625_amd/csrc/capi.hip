// C ABI of the rasteriser (declared in include/diffbmp.h): context, workspace and launches.
#include "dbmp_internal.h"
#include "diffbmp.h"
#include "workspace.h"

#include <limits.h>
#include <stdio.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>


using namespace dbmp;

static_assert(DBMP_SCHED_GRID == SCHED_GRID && DBMP_SCHED_SORTED == SCHED_SORTED &&
                  DBMP_SCHED_PERSISTENT == SCHED_PERSISTENT,
              "schedule codes of the ABI and the kernels agree");

struct dbmp_ctx {
    int device = 0;
    std::string err;
    Buf recs, tile_count, tile_len, lists, saveK, saveT, atlas_pad, box, imgs, flags, counter,
        list_max, loss_tile, order, order_hist, queue;
    int list_cap = 0;  // entries per tile list
    // launch schedule of the raster kernels (dbmp_set_schedule)
    int sched = SCHED_GRID;
    int wgs_per_cu = 4;
    int grab = 1;
    int n_cu = 256;
    int atlas_place = DBMP_ATLAS_GLOBAL;  // dbmp_set_atlas_placement
    // one-shot timing events for the next raster launch of each stage (0 forward, 1 backward)
    hipEvent_t time_ev[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    // the padded atlas held in atlas_pad (set by dbmp_set_atlas or a render given an atlas)
    bool atlas_valid = false;
    int atlas_B = 0, atlas_Hb = 0, atlas_Wb = 0, atlas_dtype = 0;
    std::vector<ImgDev> imgs_uploaded;  // what the device copy of the descriptors holds
    long long epoch = 0;                // workspace growths so far (dbmp_workspace_epoch)
    // state of the last forward, for the backward
    bool have_fwd = false;
    bool have_loss = false;
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

// Device operations of a workspace growth (workspace.h). The device is synchronised before a
// block is released: a context may have work queued on several streams (a fit's warm-up on a side
// stream, graph replays), and any of it may still read the old block.
struct HipOps {
    dbmp_ctx *c;
    const char *what;
    int quiesce()
    {
        hipError_t e = hipDeviceSynchronize();
        return e == hipSuccess ? 0 : hip_fail(c, e, "hipDeviceSynchronize");
    }
    void release(void *p) { (void)hipFree(p); }
    int acquire(void **p, size_t bytes)
    {
        if (hipMalloc(p, bytes) == hipSuccess) return 0;
        *p = nullptr;
        (void)hipGetLastError();
        return fail(c, DBMP_ENOMEM, std::string("hipMalloc failed for ") + what);
    }
    int clear(void *p, size_t bytes)
    {
        hipError_t e = hipMemset(p, 0, bytes);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        return e == hipSuccess ? 0 : hip_fail(c, e, "workspace clear");
    }
};

// Grows `b` to at least `bytes` (contents not preserved; must_be_zero: the new block is cleared).
// Synchronous; refused while the stream is being captured into a graph. A growth frees the old
// block, so graphs captured earlier on this context hold stale addresses: the workspace epoch
// counts the growths (dbmp_workspace_epoch).
int ensure(dbmp_ctx *c, Buf &b, size_t bytes, hipStream_t st, const char *what,
           bool must_be_zero = false)
{
    if (b.cap >= (bytes ? bytes : 16)) return DBMP_OK;
    if (capturing(st))
        return fail(c, DBMP_ESTATE, std::string("workspace '") + what +
                                        "' must grow during graph capture; run the call once "
                                        "before capturing");
    HipOps ops{c, what};
    bool grown = false;
    const int rc = grow_buffer(b, bytes, must_be_zero, ops, &grown);
    if (grown) ++c->epoch;
    return rc;
}

// List capacities are kept a multiple of 32 entries so every tile's list starts on its own
// 128-byte line (no two tiles share a cache line of list entries).
int round_cap(int c) { return (c + 31) & ~31; }

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

// Validates an atlas and pads it into the context (enqueued on st).
int set_atlas_impl(dbmp_ctx *c, hipStream_t st, const void *atlas, int B, int Hb, int Wb,
                   int dtype)
{
    if (!atlas || B < 1 || Hb < 2 || Wb < 2) return fail(c, DBMP_EINVAL, "bad atlas shape");
    if (dtype != DBMP_F32 && dtype != DBMP_BF16 && dtype != DBMP_F16)
        return fail(c, DBMP_EINVAL, "bad atlas dtype");
    const int Hp = Hb + 2, Wp = Wb + 2;
    const size_t esz = dtype == DBMP_F32 ? 4 : 2;
    if (!atlas_addressable(B, Hb, Wb, (long long)esz))
        return fail(c, DBMP_EINVAL, "atlas too large (the padded copy must stay below 4 GiB)");
    c->atlas_valid = false;  // until the new copy is enqueued (a failed growth frees the old one)
    int rc;
    if ((rc = ensure(c, c->atlas_pad, esz * (size_t)padded_atlas_elems(B, Hb, Wb), st, "atlas")))
        return rc;
    if ((rc = ensure(c, c->box, 16 * (size_t)B, st, "boxes"))) return rc;
    BinArgs ba{};
    ba.atlas = atlas; ba.dtype = dtype; ba.B = B; ba.Hb = Hb; ba.Wb = Wb; ba.Wp = Wp;
    ba.atlas_pad = c->atlas_pad.p; ba.box = (int *)c->box.p; ba.pad_atlas = true;
    ba.n_rows = 0;
    hipError_t e = launch_binning(ba, st);
    if (e != hipSuccess) return hip_fail(c, e, "atlas launch");
    c->atlas_valid = true;
    c->atlas_B = B; c->atlas_Hb = Hb; c->atlas_Wb = Wb; c->atlas_dtype = dtype;
    return DBMP_OK;
}

// Moves the events armed by dbmp_time_next_launch for `stage` into the launch arguments (never
// during graph capture: the events are dropped there).
void take_timing(dbmp_ctx *c, int stage, hipStream_t st, RasterArgs &a)
{
    a.ev_start = a.ev_stop = nullptr;
    if (c->time_ev[stage][0] && !capturing(st)) {
        a.ev_start = c->time_ev[stage][0];
        a.ev_stop = c->time_ev[stage][1];
    }
    c->time_ev[stage][0] = c->time_ev[stage][1] = nullptr;
}

// Shared body of dbmp_render and dbmp_render_batched. atlas == NULL: the context's atlas.
// MSE fit step fused into the forward (dbmp_render_mse): the target and the gradient buffer.
struct FuseMse {
    const float *target = nullptr;
    float *dparams = nullptr;
    bool accumulate = false;
    AdamArgs adam{};  // dbmp_fit_step: the binning first applies the pending Adam update
};

int render_impl(dbmp_ctx *c, hipStream_t st, const std::vector<dbmp_image_desc> &descs,
                const float *params, const int32_t *atlas_idx, const void *atlas, int B, int Hb,
                int Wb, int dtype, const float *bg, int bg_pp, float alpha_max, int tile,
                float *image, float *alpha, const FuseMse &fuse = FuseMse())
{
    if (!bg) return fail(c, DBMP_EINVAL, "bg is NULL");
    if (!(alpha_max > 0.f && alpha_max <= 1.f))
        return fail(c, DBMP_EINVAL, "alpha_max must be in (0, 1]");
    if (tile == 0) tile = DBMP_DEFAULT_TILE;
    if (tile != 8 && tile != 16 && tile != 32)
        return fail(c, DBMP_EINVAL, "tile must be 8, 16, 32 or 0");
    if (!image) return fail(c, DBMP_EINVAL, "image is NULL");
    int rc;
    if (atlas) {
        if (capturing(st) && !(c->atlas_valid && B == c->atlas_B && Hb == c->atlas_Hb &&
                               Wb == c->atlas_Wb && dtype == c->atlas_dtype))
            return fail(c, DBMP_ESTATE, "atlas shape changed during graph capture");
        if ((rc = set_atlas_impl(c, st, atlas, B, Hb, Wb, dtype))) return rc;
    } else if (!c->atlas_valid) {
        return fail(c, DBMP_EINVAL, "atlas is NULL and no atlas was set on this context");
    }
    B = c->atlas_B; Hb = c->atlas_Hb; Wb = c->atlas_Wb; dtype = c->atlas_dtype;
    const int Wp = Wb + 2;

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
    if (fuse.target && n_rows > 0 && !fuse.dparams)
        return fail(c, DBMP_EINVAL, "dL_dparams is NULL");
    if (n_rows >= INT_MAX) return fail(c, DBMP_EINVAL, "too many primitives");
    if ((long long)tiles * c->list_cap >= (1LL << 40))
        return fail(c, DBMP_EINVAL, "tile lists too large");

    const size_t ni = imgs.size();
    if ((rc = ensure(c, c->recs, sizeof(PrimRec) * (size_t)n_rows, st, "records"))) return rc;
    if ((rc = ensure(c, c->tile_count, 4 * (size_t)tiles, st, "tile_count", true))) return rc;
    if ((rc = ensure(c, c->tile_len, 4 * (size_t)tiles, st, "tile_len"))) return rc;
    if ((rc = ensure(c, c->loss_tile, 4 * (size_t)tiles, st, "loss_tile"))) return rc;
    if ((rc = ensure(c, c->lists, 4 * (size_t)tiles * c->list_cap, st, "tile lists"))) return rc;
    if ((rc = ensure(c, c->saveK, 4 * (size_t)n_pix, st, "saveK"))) return rc;
    if ((rc = ensure(c, c->saveT, 4 * (size_t)n_pix, st, "saveT"))) return rc;
    if (c->sched != SCHED_GRID &&
        ((rc = ensure(c, c->order, 4 * (size_t)tiles, st, "tile order")) ||
         (rc = ensure(c, c->order_hist, order_hist_bytes(tiles), st, "tile order counts"))))
        return rc;
    if (c->imgs.cap < sizeof(ImgDev) * ni || !same_imgs(imgs, c->imgs_uploaded)) {
        if (capturing(st))
            return fail(c, DBMP_ESTATE,
                        "image descriptors changed during graph capture; run the call once "
                        "before capturing");
        if ((rc = ensure(c, c->imgs, sizeof(ImgDev) * ni, st, "descriptors"))) return rc;
        // earlier launches, on any stream, may still read the table
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
        e = hipMemcpy(c->imgs.p, imgs.data(), sizeof(ImgDev) * ni, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(c, e, "descriptor upload");
        c->imgs_uploaded = imgs;
    }

    BinArgs ba{};
    ba.params = params; ba.idx = atlas_idx; ba.n_rows = n_rows;
    ba.imgs = (const ImgDev *)c->imgs.p; ba.n_images = (int)ni; ba.n_tiles = (int)tiles;
    ba.atlas = nullptr; ba.dtype = dtype; ba.B = B; ba.Hb = Hb; ba.Wb = Wb; ba.Wp = Wp;
    ba.alpha_max = alpha_max; ba.TS = tile; ba.atlas_pad = c->atlas_pad.p;
    ba.box = (int *)c->box.p; ba.recs = (PrimRec *)c->recs.p;
    ba.tile_count = (int *)c->tile_count.p; ba.lists = (int *)c->lists.p;
    ba.list_cap = c->list_cap; ba.flags = (int *)c->flags.p; ba.pad_atlas = false;
    ba.order = c->sched != SCHED_GRID ? (int *)c->order.p : nullptr;
    ba.order_hist = (int *)c->order_hist.p;
    ba.adam = fuse.adam;
    ba.prev_len = (const int *)c->tile_len.p;
    hipError_t e = launch_binning(ba, st);
    if (e != hipSuccess) return hip_fail(c, e, "binning launch");

    RasterArgs &ra = c->ra;
    ra = RasterArgs{};
    ra.recs = (const PrimRec *)c->recs.p;
    ra.lists = (const int *)c->lists.p;
    ra.list_cap = c->list_cap;
    ra.tile_count = (int *)c->tile_count.p;
    ra.tile_len = (int *)c->tile_len.p;
    ra.list_max = (int *)c->list_max.p;
    ra.imgs = (const ImgDev *)c->imgs.p;
    ra.n_images = (int)ni; ra.n_tiles = (int)tiles;
    ra.atlas_pad = c->atlas_pad.p; ra.dtype = dtype; ra.Wp = Wp; ra.Hb = Hb; ra.Wb = Wb;
    ra.zcell = (int)zero_cell(B, Hb, Wb);
    {
        const long long bytes = (dtype == DBMP_F32 ? 4LL : 2LL) * padded_atlas_elems(B, Hb, Wb);
        ra.atlas_lds_bytes =
            c->atlas_place == DBMP_ATLAS_LDS && bytes <= DBMP_ATLAS_LDS_MAX_BYTES ? (int)bytes : 0;
    }
    ra.bg = bg; ra.bg_pp = bg_pp; ra.image = image; ra.alpha = alpha;
    ra.saveK = (int *)c->saveK.p; ra.saveT = (float *)c->saveT.p;
    ra.flags = (const int *)c->flags.p; ra.TS = tile;
    ra.pair_counter = (unsigned long long *)c->counter.p;
    ra.loss_tile = (float *)c->loss_tile.p;
    ra.sched = c->sched;
    ra.grid = c->n_cu * c->wgs_per_cu;
    ra.n_cu = c->n_cu;
    ra.grab = c->grab;
    ra.order = (const int *)c->order.p;
    ra.queue = (int *)c->queue.p;
    take_timing(c, 0, st, ra);
    if (fuse.target) {  // dparams checked before anything was launched
        ra.target = fuse.target;
        ra.dparams = fuse.dparams;
        if (!fuse.accumulate && n_rows > 0) {
            e = launch_fill0(fuse.dparams, n_rows * 8, st);
            if (e != hipSuccess) return hip_fail(c, e, "gradient clear");
        }
    }
    ra.fit_state = fuse.adam.params ? fuse.adam.state : nullptr;
    e = launch_raster_fwd(ra, st);
    ra.ev_start = ra.ev_stop = nullptr;
    ra.target = nullptr;  // the saved state is that of a plain forward
    ra.dparams = nullptr;
    ra.fit_state = nullptr;
    if (e != hipSuccess) {
        // the appended counts were not consumed: clear them for the next forward
        (void)hipStreamSynchronize(st);
        (void)hipMemset(c->tile_count.p, 0, c->tile_count.cap);
        return hip_fail(c, e, "forward launch");
    }
    c->have_fwd = true;
    c->have_loss = fuse.target != nullptr;
    c->n_rows = n_rows;
    c->err.clear();
    return DBMP_OK;
}

}  // namespace

extern "C" {

int dbmp_create(dbmp_ctx **out, int device, long long list_capacity)
{
    if (!out || list_capacity < 0 || list_capacity >= (1LL << 24)) return DBMP_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return DBMP_EINVAL;
    dbmp_ctx *c = new (std::nothrow) dbmp_ctx();
    if (!c) return DBMP_ENOMEM;
    c->device = device;
    c->list_cap = round_cap(list_capacity > 0 ? (int)list_capacity : 256);
    DeviceGuard g(device);
    int rc = ensure(c, c->flags, 4 * F_COUNT, nullptr, "flags");
    if (!rc) rc = ensure(c, c->counter, 8 * DBMP_COUNTER_SLOTS, nullptr, "counter");
    if (!rc) rc = ensure(c, c->list_max, 4 * DBMP_COUNTER_SLOTS, nullptr, "list_max");
    if (!rc) rc = ensure(c, c->queue, 16, nullptr, "work queues");
    if (rc) { dbmp_destroy(c); return rc; }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) ==
            hipSuccess && ncu > 0)
        c->n_cu = ncu;
    hipError_t e = hipMemset(c->flags.p, 0, 4 * F_COUNT);
    if (e == hipSuccess) e = hipMemset(c->queue.p, 0, 16);
    if (e == hipSuccess) e = hipMemset(c->counter.p, 0, 8 * DBMP_COUNTER_SLOTS);
    if (e == hipSuccess) e = hipMemset(c->list_max.p, 0, 4 * DBMP_COUNTER_SLOTS);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) { dbmp_destroy(c); return DBMP_EHIP; }
    *out = c;
    return DBMP_OK;
}

int dbmp_destroy(dbmp_ctx *c)
{
    if (!c) return DBMP_EINVAL;
    {
        DeviceGuard g(c->device);
        (void)hipDeviceSynchronize();
        Buf *bs[] = {&c->recs, &c->tile_count, &c->tile_len, &c->lists, &c->saveK, &c->saveT,
                     &c->atlas_pad, &c->box, &c->imgs, &c->flags, &c->counter, &c->list_max,
                     &c->loss_tile, &c->order, &c->order_hist, &c->queue};
        for (Buf *b : bs)
            if (b->p) (void)hipFree(b->p);
    }
    delete c;
    return DBMP_OK;
}

int dbmp_reserve(dbmp_ctx *c, long long list_capacity)
{
    if (!c || list_capacity < 0 || list_capacity >= (1LL << 24)) return DBMP_EINVAL;
    DeviceGuard g(c->device);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(c, e, "hipDeviceSynchronize");
    if (list_capacity > c->list_cap) {
        c->list_cap = round_cap((int)list_capacity);  // the buffer grows at the next forward
        c->have_fwd = false;               // the lists of the last forward are stale
    }
    e = hipMemset(c->list_max.p, 0, 4 * DBMP_COUNTER_SLOTS);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(c, e, "statistics reset");
    return DBMP_OK;
}

int dbmp_time_next_launch(dbmp_ctx *c, int stage, void *start_event, void *stop_event)
{
    if (!c) return DBMP_EINVAL;
    if (stage != 0 && stage != 1) return fail(c, DBMP_EINVAL, "stage must be 0 or 1");
    if (!start_event != !stop_event)
        return fail(c, DBMP_EINVAL, "give both events or neither");
    c->time_ev[stage][0] = (hipEvent_t)start_event;
    c->time_ev[stage][1] = (hipEvent_t)stop_event;
    return DBMP_OK;
}

int dbmp_set_atlas_placement(dbmp_ctx *c, int placement)
{
    if (!c) return DBMP_EINVAL;
    if (placement != DBMP_ATLAS_GLOBAL && placement != DBMP_ATLAS_LDS)
        return fail(c, DBMP_EINVAL, "unknown atlas placement");
    c->atlas_place = placement;
    return DBMP_OK;
}

int dbmp_set_schedule(dbmp_ctx *c, int schedule, int workgroups_per_cu, int items_per_grab)
{
    if (!c) return DBMP_EINVAL;
    if (schedule != DBMP_SCHED_GRID && schedule != DBMP_SCHED_SORTED &&
        schedule != DBMP_SCHED_PERSISTENT)
        return fail(c, DBMP_EINVAL, "unknown schedule");
    if (workgroups_per_cu < 1 || workgroups_per_cu > 32)
        return fail(c, DBMP_EINVAL, "workgroups_per_cu must be in [1, 32]");
    if (items_per_grab < 0 || items_per_grab > 1024)
        return fail(c, DBMP_EINVAL, "items_per_grab must be in [0, 1024]");
    c->sched = schedule;
    c->wgs_per_cu = workgroups_per_cu;
    c->grab = items_per_grab;
    return DBMP_OK;
}

int dbmp_set_atlas(dbmp_ctx *c, dbmp_stream stream, const void *atlas, int B, int Hb, int Wb,
                   int atlas_dtype)
{
    if (!c) return DBMP_EINVAL;
    DeviceGuard g(c->device);
    int rc = set_atlas_impl(c, (hipStream_t)stream, atlas, B, Hb, Wb, atlas_dtype);
    if (!rc) c->err.clear();
    return rc;
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

int dbmp_render_mse(dbmp_ctx *c, dbmp_stream stream, const float *params,
                    const int32_t *atlas_idx, int N, const void *atlas, int B, int Hb, int Wb,
                    int atlas_dtype, int H, int W, const float *bg, int bg_per_pixel,
                    float alpha_max, int tile, const float *target, float *image,
                    float *dL_dparams, int accumulate)
{
    if (!c) return DBMP_EINVAL;
    if (N < 0 || H < 1 || W < 1) return fail(c, DBMP_EINVAL, "bad N / H / W");
    if (!target) return fail(c, DBMP_EINVAL, "target is NULL");
    DeviceGuard g(c->device);
    std::vector<dbmp_image_desc> d(1);
    d[0].H = H; d[0].W = W; d[0].N = N; d[0].reserved = 0;
    d[0].prim_offset = 0; d[0].pixel_offset = 0;
    FuseMse f;
    f.target = target;
    f.dparams = dL_dparams;
    f.accumulate = accumulate != 0;
    return render_impl(c, (hipStream_t)stream, d, params, atlas_idx, atlas, B, Hb, Wb,
                       atlas_dtype, bg, bg_per_pixel ? 1 : 0, alpha_max, tile, image, nullptr, f);
}

int dbmp_render_batched_mse(dbmp_ctx *c, dbmp_stream stream, int n_images,
                            const dbmp_image_desc *descs, const float *params,
                            const int32_t *atlas_idx, const void *atlas, int B, int Hb, int Wb,
                            int atlas_dtype, const float *bg, float alpha_max, int tile,
                            const float *target, float *image, float *dL_dparams, int accumulate)
{
    if (!c) return DBMP_EINVAL;
    if (n_images < 1 || !descs) return fail(c, DBMP_EINVAL, "need n_images >= 1 descriptors");
    if (!target) return fail(c, DBMP_EINVAL, "target is NULL");
    DeviceGuard g(c->device);
    std::vector<dbmp_image_desc> d(descs, descs + n_images);
    FuseMse f;
    f.target = target;
    f.dparams = dL_dparams;
    f.accumulate = accumulate != 0;
    return render_impl(c, (hipStream_t)stream, d, params, atlas_idx, atlas, B, Hb, Wb,
                       atlas_dtype, bg, 0, alpha_max, tile, image, nullptr, f);
}

namespace {
int adam_args(dbmp_ctx *c, long long n_rows, float *params, float *grad, float *m, float *v,
              int32_t *state, float lr, float beta1, float beta2, float eps, AdamArgs &a)
{
    if (!state || (n_rows > 0 && (!params || !grad || !m || !v)))
        return fail(c, DBMP_EINVAL, "params / grad / m / v / state is NULL");
    if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(c, DBMP_EINVAL, "bad Adam hyper-parameters");
    a.params = params; a.grad = grad; a.m = m; a.v = v; a.state = state;
    a.lr = lr; a.b1 = beta1; a.b2 = beta2; a.eps = eps;
    return DBMP_OK;
}
}  // namespace

int dbmp_fit_step(dbmp_ctx *c, dbmp_stream stream, float *params, const int32_t *atlas_idx,
                  int N, int H, int W, const float *bg, int bg_per_pixel, float alpha_max,
                  int tile, const float *target, float *image, float *grad, float *m, float *v,
                  int32_t *state, float lr, float beta1, float beta2, float eps)
{
    if (!c) return DBMP_EINVAL;
    if (N < 0 || H < 1 || W < 1) return fail(c, DBMP_EINVAL, "bad N / H / W");
    if (!target) return fail(c, DBMP_EINVAL, "target is NULL");
    DeviceGuard g(c->device);
    FuseMse f;
    int rc = adam_args(c, N, params, grad, m, v, state, lr, beta1, beta2, eps, f.adam);
    if (rc) return rc;
    f.target = target;
    f.dparams = grad;
    f.accumulate = true;
    std::vector<dbmp_image_desc> d(1);
    d[0].H = H; d[0].W = W; d[0].N = N; d[0].reserved = 0;
    d[0].prim_offset = 0; d[0].pixel_offset = 0;
    return render_impl(c, (hipStream_t)stream, d, params, atlas_idx, nullptr, 0, 0, 0, 0, bg,
                       bg_per_pixel ? 1 : 0, alpha_max, tile, image, nullptr, f);
}

int dbmp_fit_step_batched(dbmp_ctx *c, dbmp_stream stream, int n_images,
                          const dbmp_image_desc *descs, float *params, const int32_t *atlas_idx,
                          const float *bg, float alpha_max, int tile, const float *target,
                          float *image, float *grad, float *m, float *v, int32_t *state, float lr,
                          float beta1, float beta2, float eps)
{
    if (!c) return DBMP_EINVAL;
    if (n_images < 1 || !descs) return fail(c, DBMP_EINVAL, "need n_images >= 1 descriptors");
    if (!target) return fail(c, DBMP_EINVAL, "target is NULL");
    DeviceGuard g(c->device);
    long long rows = 0;
    for (int i = 0; i < n_images; ++i)
        rows = std::max(rows, (long long)descs[i].prim_offset + descs[i].N);
    FuseMse f;
    int rc = adam_args(c, rows, params, grad, m, v, state, lr, beta1, beta2, eps, f.adam);
    if (rc) return rc;
    f.target = target;
    f.dparams = grad;
    f.accumulate = true;
    std::vector<dbmp_image_desc> d(descs, descs + n_images);
    return render_impl(c, (hipStream_t)stream, d, params, atlas_idx, nullptr, 0, 0, 0, 0, bg, 0,
                       alpha_max, tile, image, nullptr, f);
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
    take_timing(c, 1, (hipStream_t)stream, a);
    hipError_t e = launch_raster_bwd(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "backward launch");
    c->err.clear();
    return DBMP_OK;
}

int dbmp_render_backward_mse(dbmp_ctx *c, dbmp_stream stream, const float *target,
                             const float *dL_dalpha, float *dL_dparams, int accumulate)
{
    if (!c) return DBMP_EINVAL;
    if (!c->have_fwd) return fail(c, DBMP_ESTATE, "no forward on this context");
    if (!target || (c->n_rows > 0 && !dL_dparams))
        return fail(c, DBMP_EINVAL, "target / dL_dparams is NULL");
    DeviceGuard g(c->device);
    RasterArgs a = c->ra;
    a.target = target;
    a.gA = dL_dalpha;
    a.dparams = dL_dparams;
    a.n_param_floats = accumulate ? 0 : c->n_rows * 8;  // 0: no clear before accumulating
    take_timing(c, 1, (hipStream_t)stream, a);
    hipError_t e = launch_raster_bwd(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "backward launch");
    c->have_loss = true;
    c->err.clear();
    return DBMP_OK;
}

int dbmp_mse_loss(dbmp_ctx *c, dbmp_stream stream, float *out)
{
    if (!c) return DBMP_EINVAL;
    if (!c->have_loss) return fail(c, DBMP_ESTATE, "no dbmp_render_backward_mse on this context");
    if (!out) return fail(c, DBMP_EINVAL, "out is NULL");
    DeviceGuard g(c->device);
    hipError_t e = launch_loss_sum(c->ra.loss_tile, c->ra.imgs, c->ra.n_images, out,
                                   (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "loss launch");
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
        return fail(c, DBMP_EOVERFLOW, "a tile list exceeds the capacity of " +
                                           std::to_string(c->list_cap) +
                                           " entries; see dbmp_longest_list");
    if (f[F_S_BADIDX]) return fail(c, DBMP_EINVAL, "atlas index out of range");
    if (f[F_S_NONFINITE]) return fail(c, DBMP_ENONFINITE, "non-finite parameter or texel");
    return DBMP_OK;
}

long long dbmp_longest_list(dbmp_ctx *c, dbmp_stream stream)
{
    if (!c) return -1;
    DeviceGuard g(c->device);
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return -1;
    std::vector<int> m(DBMP_COUNTER_SLOTS);
    if (hipMemcpy(m.data(), c->list_max.p, 4 * DBMP_COUNTER_SLOTS, hipMemcpyDeviceToHost) !=
        hipSuccess)
        return -1;
    return *std::max_element(m.begin(), m.end());
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

long long dbmp_workspace_epoch(const dbmp_ctx *c) { return c ? c->epoch : -1; }

long long dbmp_workspace_bytes(const dbmp_ctx *c)
{
    if (!c) return -1;
    const Buf *bufs[] = {&c->recs,      &c->tile_count, &c->tile_len,  &c->lists,
                         &c->saveK,     &c->saveT,      &c->atlas_pad, &c->box,
                         &c->imgs,      &c->flags,      &c->counter,   &c->list_max,
                         &c->loss_tile, &c->order,      &c->order_hist, &c->queue};
    long long n = 0;
    for (const Buf *b : bufs) n += (long long)b->cap;
    return n;
}

const char *dbmp_last_error(const dbmp_ctx *c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
