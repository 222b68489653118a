// The reduced-precision build of the raster kernels (Sec. 3.1.2's half-precision path, as the
// fp16 instantiation of raster_kernels.h): texels in fp16, each cell row fetched as one packed
// pair and blended in packed fp16; compositing, gradients and every sum stay in float32. All
// launch forms, in a translation unit of its own so that it compiles beside raster.hip.
#include "raster_kernels.h"

namespace dbmp {

template <int LAUNCH>
static void f16_fwd(const RasterArgs &a, hipStream_t st)
{
    switch (a.TS) {
    case 8: fwd_d1<8, _Float16, LAUNCH>(a, st); break;
    case 16: fwd_d1<16, _Float16, LAUNCH>(a, st); break;
    default: fwd_d1<32, _Float16, LAUNCH>(a, st); break;
    }
}

template <int LAUNCH>
static void f16_bwd(const RasterArgs &a, hipStream_t st)
{
    switch (a.TS) {
    case 8: bwd_d1<8, _Float16, LAUNCH>(a, st); break;
    case 16: bwd_d1<16, _Float16, LAUNCH>(a, st); break;
    default: bwd_d1<32, _Float16, LAUNCH>(a, st); break;
    }
}

hipError_t launch_raster_fwd_f16(const RasterArgs &a, hipStream_t st)
{
    if (a.n_tiles > 0) {
        if (a.sched == SCHED_PERSISTENT) f16_fwd<LAUNCH_PERSISTENT>(a, st);
        else if (pipelined(a) && a.atlas_lds_bytes > 0) f16_fwd<LAUNCH_TILE_PIPE_LDS>(a, st);
        else if (pipelined(a)) f16_fwd<LAUNCH_TILE_PIPE>(a, st);
        else f16_fwd<LAUNCH_TILE>(a, st);
    }
    return hipGetLastError();
}

hipError_t launch_raster_bwd_f16(const RasterArgs &a, hipStream_t st)
{
    if (a.n_tiles > 0) {
        if (a.sched == SCHED_PERSISTENT) f16_bwd<LAUNCH_PERSISTENT>(a, st);
        else if (pipelined(a) && a.atlas_lds_bytes > 0) f16_bwd<LAUNCH_TILE_PIPE_LDS>(a, st);
        else if (pipelined(a)) f16_bwd<LAUNCH_TILE_PIPE>(a, st);
        else f16_bwd<LAUNCH_TILE>(a, st);
    }
    return hipGetLastError();
}

}  // namespace dbmp
