// The pipelined one-tile-per-workgroup build of the raster kernels (LAUNCH_TILE_PIPE in
// raster_kernels.h, and LAUNCH_TILE_PIPE_LDS, its form with the atlas staged in LDS), in a
// translation unit of its own so that it compiles beside raster.hip.
#include "raster_kernels.h"

namespace dbmp {

hipError_t launch_raster_fwd_pipe(const RasterArgs &a, hipStream_t st)
{
    if (a.atlas_lds_bytes > 0) raster_fwd_build<LAUNCH_TILE_PIPE_LDS>(a, st);
    else raster_fwd_build<LAUNCH_TILE_PIPE>(a, st);
    return hipGetLastError();
}

hipError_t launch_raster_bwd_pipe(const RasterArgs &a, hipStream_t st)
{
    if (a.atlas_lds_bytes > 0) raster_bwd_build<LAUNCH_TILE_PIPE_LDS>(a, st);
    else raster_bwd_build<LAUNCH_TILE_PIPE>(a, st);
    return hipGetLastError();
}

}  // namespace dbmp
