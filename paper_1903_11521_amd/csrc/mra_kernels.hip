// The MADNESS separable contraction (Sec. 7, Eq. stock_mra) on the matrix
// cores: for a batch of p x p x p tensors S sharing three low-rank operator
// pairs,
//     R_ijk = sum S_xyz X^L_xl X^R_li Y^L_ym Y^R_mj Z^L_zn Z^R_nk,
// evaluated as the paper's chain of six one-index contractions (x, l, y, m,
// z, n).  One workgroup (4 waves) per tensor; the tensor and its
// intermediates stay in LDS (two buffers of p^3 values); each contraction is
// a GEMM on v_mfma_f64_16x16x4f64 (FP64) or v_mfma_f32_16x16x4f32 (FP32).
//
// A contraction maps in[a][k][b] (pre, K, post) to
//     out[a][m][b] = sum_k F[k][m] in[a][k][b]
// with F the K x M factor (row major, in global memory, L1/L2 resident).
// With post >= 16 every slice a is a GEMM  out[a] = F^T in[a]  (the factor
// is the A operand, the slice the B operand); with post = 1 (the last index)
// it is one GEMM  out = in F  over all slices (the tensor rows are the A
// operand).  MFMA lane layout (16 x 16 x 4): A[i][k] in lane k*16 + i,
// B[k][j] in lane k*16 + j; output register r of a lane holds column
// lane%16 of row 4*(lane/16)+r in FP32 but of row lane/16+4r in FP64.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dgr {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Acc;
template <>
struct Acc<double> {
    typedef d4 v;
    static __device__ __forceinline__ v mfma(double a, double b, v c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
};
template <>
struct Acc<float> {
    typedef f4 v;
    static __device__ __forceinline__ v mfma(float a, float b, v c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

// One contraction step over the whole tensor, work items dealt to the 4
// waves of the workgroup.
template <typename T>
__device__ __forceinline__ void contract(const T *__restrict__ in, T *__restrict__ out, const T *__restrict__ F,
                                         int pre, int K, int M, int post)
{
    using V = typename Acc<T>::v;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int KS = (K + 3) / 4;
    if (post > 1) {
        const int MT = (M + 15) / 16, NT = (post + 15) / 16;
        const int items = pre * MT * NT;
        for (int it = wave; it < items; it += 4) {
            const int a = it / (MT * NT), rem = it - a * MT * NT;
            const int mt = rem / NT, nt = rem - mt * NT;
            const int m = mt * 16 + li, n = nt * 16 + li;
            const T *ia = in + (size_t)a * K * post;
            V c = {0, 0, 0, 0};
            for (int s = 0; s < KS; ++s) {
                const int k = 4 * s + lk;
                const T av = (k < K && m < M) ? F[k * M + m] : T(0);         // A = F^T: [m][k]
                const T bv = (k < K && n < post) ? ia[k * post + n] : T(0);  // B = in[a]: [k][n]
                c = Acc<T>::mfma(av, bv, c);
            }
            T *oa = out + (size_t)a * M * post;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int mo = mt * 16 + Acc<T>::row(lk, r);
                if (mo < M && n < post) oa[mo * post + n] = c[r];
            }
        }
    } else {
        const int AT = (pre + 15) / 16, MT = (M + 15) / 16;
        const int items = AT * MT;
        for (int it = wave; it < items; it += 4) {
            const int at = it / MT, mt = it - at * MT;
            const int a = at * 16 + li, m = mt * 16 + li;
            V c = {0, 0, 0, 0};
            for (int s = 0; s < KS; ++s) {
                const int k = 4 * s + lk;
                const T av = (k < K && a < pre) ? in[(size_t)a * K + k] : T(0);  // A = in: [a][k]
                const T bv = (k < K && m < M) ? F[k * M + m] : T(0);            // B = F: [k][m]
                c = Acc<T>::mfma(av, bv, c);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ao = at * 16 + Acc<T>::row(lk, r);
                if (ao < pre && m < M) out[(size_t)ao * M + m] = c[r];
            }
        }
    }
}

// One tensor per workgroup of 256 threads; dynamic LDS of 2 p^3 values.
template <typename T>
__global__ void __launch_bounds__(256)
k_mra(int64_t nb, int p, int q, const T *__restrict__ S, const T *__restrict__ XL, const T *__restrict__ XR,
      const T *__restrict__ YL, const T *__restrict__ YR, const T *__restrict__ ZL, const T *__restrict__ ZR,
      T *__restrict__ R)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *b0 = reinterpret_cast<T *>(lds_raw);
    const int p3 = p * p * p;
    T *b1 = b0 + p3;
    const int64_t t = blockIdx.x;
    if (t >= nb) return;
    const T *src = S + (size_t)t * p3;
    for (int i = threadIdx.x; i < p3; i += 256) b0[i] = src[i];
    __syncthreads();
    // x: [x][y z] -> [l][y z];  l: [l][y z] -> [i][y z]
    contract<T>(b0, b1, XL, 1, p, q, p * p);
    __syncthreads();
    contract<T>(b1, b0, XR, 1, q, p, p * p);
    __syncthreads();
    // y: [i][y][z] -> [i][m][z];  m: -> [i][j][z]
    contract<T>(b0, b1, YL, p, p, q, p);
    __syncthreads();
    contract<T>(b1, b0, YR, p, q, p, p);
    __syncthreads();
    // z: [i j][z] -> [i j][n];  n: -> [i j][k]
    contract<T>(b0, b1, ZL, p * p, p, q, 1);
    __syncthreads();
    contract<T>(b1, b0, ZR, p * p, q, p, 1);
    __syncthreads();
    T *dst = R + (size_t)t * p3;
    for (int i = threadIdx.x; i < p3; i += 256) dst[i] = b0[i];
}

}  // namespace dgr

// Host launcher: 0 on success, a hipError_t otherwise.
hipError_t dg_mra_launch(bool fp64, int64_t nb, int p, int q, const void *S, const void *XL, const void *XR,
                         const void *YL, const void *YR, const void *ZL, const void *ZR, void *R, hipStream_t s)
{
    if (nb == 0) return hipSuccess;
    const size_t lds = 2 * (size_t)p * p * p * (fp64 ? 8 : 4);
    // more than the default 64 KB of dynamic LDS must be allowed per kernel
    hipError_t e = fp64 ? hipFuncSetAttribute((const void *)dgr::k_mra<double>,
                                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
                        : hipFuncSetAttribute((const void *)dgr::k_mra<float>,
                                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (fp64) {
        hipLaunchKernelGGL(dgr::k_mra<double>, dim3((unsigned)nb), dim3(256), lds, s, nb, p, q,
                           (const double *)S, (const double *)XL, (const double *)XR, (const double *)YL,
                           (const double *)YR, (const double *)ZL, (const double *)ZR, (double *)R);
    } else {
        hipLaunchKernelGGL(dgr::k_mra<float>, dim3((unsigned)nb), dim3(256), lds, s, nb, p, q,
                           (const float *)S, (const float *)XL, (const float *)XR, (const float *)YL,
                           (const float *)YR, (const float *)ZL, (const float *)ZR, (float *)R);
    }
    return hipGetLastError();
}
