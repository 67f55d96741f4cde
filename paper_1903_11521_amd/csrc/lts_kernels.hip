// Element-wise kernels of clustered local time stepping (rate 2): the ghost
// face-trace slots a cluster's corrector reads for its neighbours in other
// clusters, and the trace buffer of a smaller cluster's steps.  The ADER
// stages themselves are the step kernels.  real = double or float; base
// pointers are such that p + v * TB is element v's slot.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lts_internal.h"

namespace dgl {

// One thread per value (n TB < 2^31, checked by the launcher).
template <typename real>
__global__ void __launch_bounds__(256)
k_ghosts(int total, int TB, const int32_t *__restrict__ ids, const int8_t *__restrict__ kind, int half,
         const real *__restrict__ up_tr, const real *__restrict__ half_tr, const real *__restrict__ buf_tr,
         real *__restrict__ dst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int g = i / TB, r = i - g * TB;
    const int64_t o = (int64_t)ids[g] * TB + r;
    real out;
    if (kind[g] == 2) out = buf_tr[o];
    else if (half == 0) out = half_tr[o];
    else out = up_tr[o] - half_tr[o];
    dst[(int64_t)g * TB + r] = out;
}

template <typename real>
__global__ void __launch_bounds__(256)
k_tbuffer(int total, int TB, const int32_t *__restrict__ ids, const real *__restrict__ src_tr,
          real *__restrict__ buf_tr, int reset)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int j = i / TB, r = i - j * TB;
    const int64_t o = (int64_t)ids[j] * TB + r;
    buf_tr[o] = reset ? src_tr[o] : buf_tr[o] + src_tr[o];
}

}  // namespace dgl

hipError_t dg_lts_ghosts(bool fp64, int64_t n, int TB, const int32_t *ids, const int8_t *kind, int half,
                         const void *up_tr, const void *half_tr, const void *buf_tr, void *dst, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (n * TB > 0x7fffffff) return hipErrorInvalidValue;
    const int total = (int)(n * TB);
    const dim3 grid((unsigned)((total + 255) / 256));
    if (fp64)
        hipLaunchKernelGGL(dgl::k_ghosts<double>, grid, dim3(256), 0, s, total, TB, ids, kind, half,
                           (const double *)up_tr, (const double *)half_tr, (const double *)buf_tr, (double *)dst);
    else
        hipLaunchKernelGGL(dgl::k_ghosts<float>, grid, dim3(256), 0, s, total, TB, ids, kind, half,
                           (const float *)up_tr, (const float *)half_tr, (const float *)buf_tr, (float *)dst);
    return hipGetLastError();
}

hipError_t dg_lts_tbuffer(bool fp64, int64_t n, int TB, const int32_t *ids, const void *src_tr, void *buf_tr,
                          bool reset, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (n * TB > 0x7fffffff) return hipErrorInvalidValue;
    const int total = (int)(n * TB);
    const dim3 grid((unsigned)((total + 255) / 256));
    if (fp64)
        hipLaunchKernelGGL(dgl::k_tbuffer<double>, grid, dim3(256), 0, s, total, TB, ids, (const double *)src_tr,
                           (double *)buf_tr, reset ? 1 : 0);
    else
        hipLaunchKernelGGL(dgl::k_tbuffer<float>, grid, dim3(256), 0, s, total, TB, ids, (const float *)src_tr,
                           (float *)buf_tr, reset ? 1 : 0);
    return hipGetLastError();
}
