// Element-wise kernels of clustered local time stepping (rate 2): the
// neighbour-integral gather and the buffer of a smaller cluster's step
// integrals.  The ADER stages themselves are the per-stage kernels.
//
// Layouts (storage type real = double or float, PB = 9 B values per
// element): T [E][N+1][PB] Taylor-scaled derivatives T^d = dt^d/d! D^d of
// each element's latest predictor (scaled with its own cluster's dt);
// I, Buf, G [E][PB].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lts_internal.h"

namespace dgl {

// G[v] for the listed elements v = ids[j]:
//   kind 0: I[v]                                 (same cluster as the receiver)
//   kind 1: sum_d w[d] T[v][d], w[d] = dt (b^(d+1) - a^(d+1)) / (d+1)
//                                                (larger neighbour; the receiver's
//                                                 interval [a, b] dt inside its step)
//   kind 2: Buf[v]                               (smaller neighbour: its step
//                                                 integrals summed over the receiver's
//                                                 interval)
// One workgroup per listed element; FP64 accumulation of the sub-interval sum.
template <typename real>
__global__ void __launch_bounds__(256)
k_gather(int PB, int N1, const int32_t *__restrict__ ids, const int8_t *__restrict__ kind,
         const real *__restrict__ T, const real *__restrict__ I, const real *__restrict__ Buf,
         real *__restrict__ G, LtsWeights w)
{
    const int64_t v = ids[blockIdx.x];
    const int k = kind[blockIdx.x];
    real *g = G + v * PB;
    if (k == 0) {
        const real *src = I + v * PB;
        for (int r = threadIdx.x; r < PB; r += blockDim.x) g[r] = src[r];
    } else if (k == 2) {
        const real *src = Buf + v * PB;
        for (int r = threadIdx.x; r < PB; r += blockDim.x) g[r] = src[r];
    } else {
        const real *t = T + v * N1 * PB;
        for (int r = threadIdx.x; r < PB; r += blockDim.x) {
            double s = 0.0;
            for (int d = 0; d < N1; ++d) s = fma(w.w[d], (double)t[d * PB + r], s);
            g[r] = (real)s;
        }
    }
}

// Buf[v] = I[v] (reset) or Buf[v] + I[v] for the listed elements.
template <typename real>
__global__ void __launch_bounds__(256)
k_buffer(int PB, const int32_t *__restrict__ ids, const real *__restrict__ I, real *__restrict__ Buf, int reset)
{
    const int64_t v = ids[blockIdx.x];
    const real *src = I + v * PB;
    real *dst = Buf + v * PB;
    if (reset) {
        for (int r = threadIdx.x; r < PB; r += blockDim.x) dst[r] = src[r];
    } else {
        for (int r = threadIdx.x; r < PB; r += blockDim.x) dst[r] = (real)((double)dst[r] + (double)src[r]);
    }
}

}  // namespace dgl

hipError_t dg_lts_gather(bool fp64, int64_t n, int PB, int N1, const int32_t *ids, const int8_t *kind,
                         const void *T, const void *I, const void *Buf, void *G, const LtsWeights &w, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(dgl::k_gather<double>, dim3((unsigned)n), dim3(256), 0, s, PB, N1, ids, kind,
                           (const double *)T, (const double *)I, (const double *)Buf, (double *)G, w);
    else
        hipLaunchKernelGGL(dgl::k_gather<float>, dim3((unsigned)n), dim3(256), 0, s, PB, N1, ids, kind,
                           (const float *)T, (const float *)I, (const float *)Buf, (float *)G, w);
    return hipGetLastError();
}

hipError_t dg_lts_buffer(bool fp64, int64_t n, int PB, const int32_t *ids, const void *I, void *Buf, bool reset,
                         hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(dgl::k_buffer<double>, dim3((unsigned)n), dim3(256), 0, s, PB, ids, (const double *)I,
                           (double *)Buf, reset ? 1 : 0);
    else
        hipLaunchKernelGGL(dgl::k_buffer<float>, dim3((unsigned)n), dim3(256), 0, s, PB, ids, (const float *)I,
                           (float *)Buf, reset ? 1 : 0);
    return hipGetLastError();
}
