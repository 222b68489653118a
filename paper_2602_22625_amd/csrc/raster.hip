// Raster launches (Sec. 3.1.1-3.1.2; Supp. Eqs. S1-S5): the kernels are in raster_kernels.h.
// This file builds the one-tile-per-workgroup and persistent forms; raster_pipe.hip builds the
// pipelined one-tile-per-workgroup form and raster_f16.hip every form of the fp16 build
// (separate translation units, compiled in parallel).
#include "raster_kernels.h"

namespace dbmp {

__global__ void k_fill0(float *__restrict__ p, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// Per-image sums of the per-tile squared errors: one workgroup per image, out[image].
__global__ void __launch_bounds__(256) k_loss_sum(const float *__restrict__ lt,
                                                  const ImgDev *__restrict__ imgs,
                                                  float *__restrict__ out)
{
    const ImgDev D = imgs[blockIdx.x];
    const int nt = D.ntx * D.nty;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nt; i += 256) acc += lt[D.tile_off + i];
    __shared__ double s[256];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = (float)s[0];
}

hipError_t launch_raster_fwd(const RasterArgs &a, hipStream_t st)
{
    if (a.dtype == 2) return launch_raster_fwd_f16(a, st);
    if (a.n_tiles > 0) {
        if (a.sched == SCHED_PERSISTENT) raster_fwd_build<LAUNCH_PERSISTENT>(a, st);
        else if (pipelined(a)) return launch_raster_fwd_pipe(a, st);
        else raster_fwd_build<LAUNCH_TILE>(a, st);
    }
    return hipGetLastError();
}

hipError_t launch_raster_bwd(const RasterArgs &a, hipStream_t st)
{
    if (a.n_param_floats > 0)
        k_fill0<<<(unsigned)((a.n_param_floats + 255) / 256), 256, 0, st>>>(a.dparams,
                                                                             a.n_param_floats);
    if (a.dtype == 2) return launch_raster_bwd_f16(a, st);
    if (a.n_tiles > 0) {
        if (a.sched == SCHED_PERSISTENT) raster_bwd_build<LAUNCH_PERSISTENT>(a, st);
        else if (pipelined(a)) return launch_raster_bwd_pipe(a, st);
        else raster_bwd_build<LAUNCH_TILE>(a, st);
    }
    return hipGetLastError();
}

hipError_t launch_fill0(float *p, long long n, hipStream_t st)
{
    if (n > 0) k_fill0<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_loss_sum(const float *loss_tile, const ImgDev *imgs, int n_images, float *out,
                           hipStream_t st)
{
    k_loss_sum<<<n_images, 256, 0, st>>>(loss_tile, imgs, out);
    return hipGetLastError();
}

}  // namespace dbmp
