// Loss gradient and optimiser step (the `mse` loss and Adam optimiser of the paper's
// configuration, Supp. Table S1; here with a flat learning rate). Both are HBM-bound streams.
#include "dbmp_internal.h"
#include "diffbmp.h"

namespace dbmp {

__global__ void __launch_bounds__(256)
k_mse_grad(const float4 *__restrict__ img, const float4 *__restrict__ tgt, long long n4,
           const float *__restrict__ img1, const float *__restrict__ tgt1, long long n,
           float *__restrict__ grad, float scale, float *__restrict__ loss_sum)
{
    float acc = 0.f;
    const long long stride = (long long)gridDim.x * blockDim.x;
    float4 *g4 = (float4 *)grad;
    constexpr int U = 4;  // float4 loads in flight per thread
    for (long long i0 = (long long)blockIdx.x * blockDim.x + threadIdx.x; i0 < n4;
         i0 += U * stride) {
        float4 a[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long i = i0 + u * stride;
            if (i < n4) { a[u] = img[i]; b[u] = tgt[i]; }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long i = i0 + u * stride;
            if (i >= n4) continue;
            const float4 d = make_float4(a[u].x - b[u].x, a[u].y - b[u].y, a[u].z - b[u].z,
                                         a[u].w - b[u].w);
            g4[i] = make_float4(scale * d.x, scale * d.y, scale * d.z, scale * d.w);
            acc = fmaf(d.x, d.x, acc); acc = fmaf(d.y, d.y, acc);
            acc = fmaf(d.z, d.z, acc); acc = fmaf(d.w, d.w, acc);
        }
    }
    for (long long i = 4 * n4 + (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += stride) {
        const float d = img1[i] - tgt1[i];
        grad[i] = scale * d;
        acc = fmaf(d, d, acc);
    }
    if (!loss_sum) return;
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    __shared__ float ws[4];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        // loss_sum[2] accumulates the block sums, loss_sum[1] counts finished blocks; the last
        // block publishes the total in loss_sum[0] and re-arms both for the next call
        unsafeAtomicAdd(loss_sum + 2, ws[0] + ws[1] + ws[2] + ws[3]);
        __threadfence();
        unsigned int *cnt = (unsigned int *)(loss_sum + 1);
        if (atomicAdd(cnt, 1u) == gridDim.x - 1) {
            __threadfence();
            loss_sum[0] = __hip_atomic_load(loss_sum + 2, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
            loss_sum[2] = 0.f;
            *cnt = 0u;
            __threadfence();
        }
    }
}

constexpr int ADAM_PER_THREAD = 4;

__global__ void __launch_bounds__(256)
k_adam(float *__restrict__ p, float *__restrict__ g, float *__restrict__ m,
       float *__restrict__ v, long long n, float lr, float b1, float b2, float eps,
       int *__restrict__ step, unsigned int *__restrict__ done, int zero_grad)
{
    const int t = *step + 1;
    // bias corrections 1 - beta^t, evaluated in float64 once per workgroup (a float64 pow costs
    // a wave hundreds of instructions; per element it dominated the kernel)
    __shared__ float s_c[2];
    if (threadIdx.x == 0) {
        s_c[0] = (float)(1.0 - pow((double)b1, (double)t));
        s_c[1] = (float)(1.0 - pow((double)b2, (double)t));
    }
    __syncthreads();
    const float c1 = s_c[0], c2 = s_c[1];
    const long long base = (long long)blockIdx.x * (blockDim.x * ADAM_PER_THREAD);
#pragma unroll
    for (int u = 0; u < ADAM_PER_THREAD; ++u) {
        const long long i = base + (long long)u * blockDim.x + threadIdx.x;
        if (i >= n) break;
        const float gi = g[i];
        if (zero_grad) g[i] = 0.f;  // ready for the next accumulating backward
        const float mi = fmaf(b1, m[i], (1.f - b1) * gi);
        const float vi = fmaf(b2, v[i], (1.f - b2) * gi * gi);
        m[i] = mi;
        v[i] = vi;
        const float mhat = mi / c1, vhat = vi / c2;
        p[i] = p[i] - lr * mhat / (sqrtf(vhat) + eps);
    }
    // The last block to finish advances the step counter and re-arms the completion counter
    // for the next call. Every block read the step counter (and consumed the value) before its
    // barrier and counts itself done after it, so the last block writes after every read. No
    // fence: nothing else flows between blocks, and on gfx950 a device-scope fence writes back
    // the L2 (once per block it would dominate this kernel).
    __syncthreads();
    if (threadIdx.x == 0 &&
        __hip_atomic_fetch_add(done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
            gridDim.x - 1) {
        *step = t;
        *done = 0u;
    }
}

}  // namespace dbmp

using namespace dbmp;

extern "C" int dbmp_mse_grad(dbmp_stream stream, const float *image, const float *target,
                             long long n, float *grad, float *loss_sum)
{
    if (n < 0 || (n > 0 && (!image || !target || !grad))) return DBMP_EINVAL;
    if (n == 0) return DBMP_OK;
    hipStream_t st = (hipStream_t)stream;
    const bool aligned = (((uintptr_t)image | (uintptr_t)target | (uintptr_t)grad) & 15) == 0;
    const long long n4 = aligned ? n / 4 : 0;
    long long blocks = (n + 4095) / 4096;
    if (blocks > 256) blocks = 256;
    k_mse_grad<<<(unsigned)blocks, 256, 0, st>>>((const float4 *)image, (const float4 *)target,
                                                 n4, image, target, n, grad, 2.0f / (float)n,
                                                 loss_sum);
    return hipGetLastError() == hipSuccess ? DBMP_OK : DBMP_EHIP;
}

extern "C" int dbmp_adam_step(dbmp_stream stream, float *params, float *grad, float *m,
                              float *v, long long n, float lr, float beta1, float beta2,
                              float eps, int32_t *step, int zero_grad)
{
    if (n < 0 || !step || (n > 0 && (!params || !grad || !m || !v))) return DBMP_EINVAL;
    if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return DBMP_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const long long per_block = 256LL * ADAM_PER_THREAD;
    k_adam<<<(unsigned)(n > 0 ? (n + per_block - 1) / per_block : 1), 256, 0, st>>>(
        params, grad, m, v, n, lr, beta1, beta2, eps, step, (unsigned int *)(step + 1),
        zero_grad);
    return hipGetLastError() == hipSuccess ? DBMP_OK : DBMP_EHIP;
}
