// The MADNESS separable contraction (Sec. 7, Eq. stock_mra) on the matrix
// cores: for a batch of p x p x p tensors S sharing three low-rank operator
// pairs,
//     R_ijk = sum S_xyz X^L_xl X^R_li Y^L_ym Y^R_mj Z^L_zn Z^R_nk,
// evaluated as the paper's chain of six one-index contractions (x, l, y, m,
// z, n) in FP64 (v_mfma_f64_16x16x4f64) or FP32 (v_mfma_f32_16x16x4f32).
//
// A workgroup takes blocks of T tensors (T p^3 values fill about 32 KB); a
// block and its intermediates stay in LDS (two buffers) and the six factors
// sit there too, zero padded to whole 4 x 16 MFMA fragments.  A contraction
// maps in[a][k][b] (a < pre, k < K, b < post) with the K x M factor F to
//   mode "in place":  out[a][m][b] = sum_k F[k][m] in[a][k][b]   (C = F^T in)
//   mode "to last":   out[a][b][m] = sum_k in[a][k][b] F[k][m]   (C = in^T F)
// and the pair (a, b) is flattened into one MFMA tile index c, so tiles are
// never padded along a or b.  With the sequence
//   x->l, l->i, y->m in place  ([t][i][m][z]),  m->j to last ([t][i][z][j]),
//   z->n in place ([t][i][n][j]),  n->k to last ([t][i][j][k])
// every LDS read of the tensor is contiguous along the 16 lanes of a
// fragment row, and the last step writes R coalesced straight to global
// memory.  The size p is a template parameter (all index arithmetic by
// constants, LDS offsets as instruction immediates); a wave keeps the factor
// fragments of a contraction in registers and reads each tensor fragment
// once for all column blocks of the factor.
//
// MFMA lane layout (16 x 16 x 4): A[i][k] in lane 16k + i, B[k][j] in lane
// 16k + j; output register r of a lane holds column lane%16 of row
// 4(lane/16) + r in FP32 but of row lane/16 + 4r in FP64.
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
    // row of output register r is row0(lk) + r * rstep
    static constexpr int rmul = 1, rstep = 4;
};
template <>
struct Acc<float> {
    typedef f4 v;
    static __device__ __forceinline__ v mfma(float a, float b, v c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static constexpr int rmul = 4, rstep = 1;
};

constexpr int THREADS = 1024;
constexpr int WAVES = THREADS / 64;

__host__ __device__ constexpr int ks_of(int K) { return (K + 3) / 4; }
__host__ __device__ constexpr int mt_of(int M) { return (M + 15) / 16; }
// a zero-padded K x M factor: 4 KS rows of 16 MT columns
__host__ __device__ constexpr int fac_size(int K, int M) { return 4 * ks_of(K) * 16 * mt_of(M); }

// One contraction over the block.  PQ: K = P, M = q (else K = q, M = P);
// POST: the size of the trailing index b; TO_LAST: the output placement.
// out is LDS, or global memory for the last step (same indexing).
template <typename T, int P, bool PQ, int POST, bool TO_LAST>
__device__ __forceinline__ void contract(const T *__restrict__ in, T *__restrict__ out, const T *__restrict__ Fl,
                                         int q, int pre)
{
    using V = typename Acc<T>::v;
    constexpr int KSX = ks_of(P), MTX = mt_of(P);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int K = PQ ? P : q, M = PQ ? q : P;
    const int KS = PQ ? KSX : ks_of(q), MT = PQ ? mt_of(q) : MTX;
    const int Mp = 16 * MT;
    // factor fragments: F[4s + lk][16 mt + li]
    T fv[MTX][KSX];
#pragma unroll
    for (int mt = 0; mt < MTX; ++mt)
#pragma unroll
        for (int s = 0; s < KSX; ++s)
            fv[mt][s] = (mt < MT && s < KS) ? Fl[(4 * s + lk) * Mp + 16 * mt + li] : T(0);
    // rows k >= K of the last tensor fragment are not read (zero)
    const bool lastok = lk < K - 4 * (KS - 1);
    const int cols = pre * POST, CT = (cols + 15) / 16;
    for (int ct = wave; ct < CT; ct += WAVES) {
        const int c = 16 * ct + li;
        const int cc = c < cols ? c : cols - 1;            // clamped read, result discarded
        const int a = cc / POST, b = cc - a * POST;
        const T *src = in + (a * K + lk) * POST + b;
        T tv[KSX];
#pragma unroll
        for (int s = 0; s < KSX; ++s)
            tv[s] = (s < KS - 1 || (s == KS - 1 && lastok)) ? src[4 * s * POST] : T(0);
#pragma unroll
        for (int mt = 0; mt < MTX; ++mt) {
            if (mt >= MT) break;
            V acc = {0, 0, 0, 0};
#pragma unroll
            for (int s = 0; s < KSX; ++s)
                if (s < KS)
                    acc = TO_LAST ? Acc<T>::mfma(tv[s], fv[mt][s], acc)    // A = in^T [c][k], B = F [k][m]
                                  : Acc<T>::mfma(fv[mt][s], tv[s], acc);   // A = F^T [m][k], B = in [k][c]
            if (TO_LAST) {
                // C[c][m] -> out[c * P + m]
                const int m = 16 * mt + li;
                const int r0 = 16 * ct + Acc<T>::rmul * lk;
                T *o = out + r0 * P + m;
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (r0 + r * Acc<T>::rstep < cols && m < P) o[r * Acc<T>::rstep * P] = acc[r];
            } else {
                // C[m][c] -> out[a][m][b]
                const int m0 = 16 * mt + Acc<T>::rmul * lk;
                T *o = out + (a * M + m0) * POST + b;
                if (c < cols) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (m0 + r * Acc<T>::rstep < M) o[r * Acc<T>::rstep * POST] = acc[r];
                }
            }
        }
    }
}

// Stages the six factors zero padded: X^L (p x q) at 0, X^R (q x p) after
// it, then the Y and Z pairs the same way.
template <typename T, int P>
__device__ __forceinline__ void stage_factors(T *__restrict__ fl, const T *const *F, int q)
{
    constexpr int U = (3 * 2 * fac_size(P, P) + THREADS - 1) / THREADS;
    const int sp = fac_size(P, q), sq = fac_size(q, P), pair_size = sp + sq, total = 3 * pair_size;
    const int mp_pq = 16 * mt_of(q);
    constexpr int mp_qp = 16 * mt_of(P);
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        int i = threadIdx.x + u * THREADS;
        v[u] = T(0);
        if (i < total) {
            const int pair = i / pair_size;
            i -= pair * pair_size;
            const bool right = i >= sp;
            if (right) i -= sp;
            const int Mp = right ? mp_qp : mp_pq, K = right ? q : P, M = right ? P : q;
            const int k = i / Mp, m = i - k * Mp;
            if (k < K && m < M) v[u] = F[2 * pair + (right ? 1 : 0)][k * M + m];
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int i = threadIdx.x + u * THREADS;
        if (i < total) fl[i] = v[u];
    }
}

// Tensors per block: as many as fill about 32 KB per buffer.
__host__ __device__ constexpr int mra_tpb(int p, int elem)
{
    return 32768 / (p * p * p * elem) < 1 ? 1 : 32768 / (p * p * p * elem);
}

// Dynamic LDS: two buffers of TPB p^3 values, then the six padded factors.
// Persistent: a workgroup takes blocks blockIdx.x, + gridDim.x, ...; the
// tensors of its next block are loaded into registers while the six
// contractions of the current one run.
template <typename T, int P>
__global__ void __launch_bounds__(THREADS)
k_mra(int64_t nb, int q, const T *__restrict__ S, const T *__restrict__ XL, const T *__restrict__ XR,
      const T *__restrict__ YL, const T *__restrict__ YR, const T *__restrict__ ZL, const T *__restrict__ ZR,
      T *__restrict__ R)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    constexpr int P3 = P * P * P;
    constexpr int TPB = mra_tpb(P, (int)sizeof(T));
    constexpr int U = (TPB * P3 + THREADS - 1) / THREADS;
    const int64_t nblk = (nb + TPB - 1) / TPB;
    int64_t blk = blockIdx.x;
    if (blk >= nblk) return;
    T *b0 = reinterpret_cast<T *>(lds_raw);
    T *b1 = b0 + TPB * P3;
    T *fl = b1 + TPB * P3;
    const int sp = fac_size(P, q), sq = fac_size(q, P);
    T *fxl = fl, *fxr = fxl + sp, *fyl = fxr + sq, *fyr = fyl + sp, *fzl = fyr + sq, *fzr = fzl + sp;
    const T *const facs[6] = {XL, XR, YL, YR, ZL, ZR};
    stage_factors<T, P>(fl, facs, q);
    T v[U];
    auto fetch = [&](int64_t bk) {
        const int64_t t0 = bk * TPB;
        const int n = (int)((nb - t0) < TPB ? (nb - t0) : TPB) * P3;
        const T *src = S + t0 * P3;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = threadIdx.x + u * THREADS;
            v[u] = i < n ? __builtin_nontemporal_load(src + i) : T(0);
        }
    };
    fetch(blk);
    for (; blk < nblk; blk += gridDim.x) {
        const int64_t t0 = blk * TPB;
        const int nt = (int)((nb - t0) < TPB ? (nb - t0) : TPB);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = threadIdx.x + u * THREADS;
            if (i < nt * P3) b0[i] = v[u];
        }
        if (blk + gridDim.x < nblk) fetch(blk + gridDim.x);
        __syncthreads();
        contract<T, P, true, P * P, false>(b0, b1, fxl, q, nt);           // [t][x][yz] -> [t][l][yz]
        __syncthreads();
        contract<T, P, false, P * P, false>(b1, b0, fxr, q, nt);          // -> [t][i][y][z]
        __syncthreads();
        contract<T, P, true, P, false>(b0, b1, fyl, q, nt * P);           // [ti][y][z] -> [ti][m][z]
        __syncthreads();
        contract<T, P, false, P, true>(b1, b0, fyr, q, nt * P);           // [ti][m][z] -> [ti][z][j]
        __syncthreads();
        contract<T, P, true, P, false>(b0, b1, fzl, q, nt * P);           // [ti][z][j] -> [ti][n][j]
        __syncthreads();
        contract<T, P, false, P, true>(b1, R + t0 * P3, fzr, q, nt * P);  // -> [ti][j][k]
        // the next block's stores into b0 follow the last reads of b0 (the
        // z -> n step, before the barrier above); its first contraction
        // writes b1 only after the barrier that follows those stores
    }
}

template <typename T, int P>
hipError_t launch_p(int64_t nb, int q, const void *S, const void *XL, const void *XR, const void *YL,
                    const void *YR, const void *ZL, const void *ZR, void *R, hipStream_t s)
{
    constexpr int TPB = mra_tpb(P, (int)sizeof(T));
    const size_t lds = (2 * (size_t)TPB * P * P * P + 3 * (size_t)(fac_size(P, q) + fac_size(q, P))) * sizeof(T);
    // per thread and instantiation: the last device and LDS size seen, with
    // the CU count and the resident workgroups per CU found for them
    static thread_local int c_dev = -1, c_cus = 0, c_per_cu = 0;
    static thread_local size_t c_lds = 0;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev != c_dev || lds != c_lds) {
        // more than the default 64 KB of dynamic LDS must be allowed per kernel
        if ((e = hipFuncSetAttribute((const void *)k_mra<T, P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds)) != hipSuccess)
            return e;
        int cus = 0, per_cu = 0;
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_mra<T, P>, THREADS, lds)) !=
            hipSuccess)
            return e;
        c_dev = dev, c_lds = lds, c_cus = cus, c_per_cu = per_cu < 1 ? 1 : per_cu;
    }
    const int cus = c_cus, per_cu = c_per_cu;
    const int64_t nblk = (nb + TPB - 1) / TPB, cap = (int64_t)cus * per_cu;
    const unsigned grid = (unsigned)(nblk < cap ? nblk : cap);
    hipLaunchKernelGGL((k_mra<T, P>), dim3(grid), dim3(THREADS), lds, s, nb, q, (const T *)S, (const T *)XL,
                       (const T *)XR, (const T *)YL, (const T *)YR, (const T *)ZL, (const T *)ZR, (T *)R);
    return hipGetLastError();
}

template <typename T, int P>
struct Dispatch {
    static hipError_t run(int p, int64_t nb, int q, const void *S, const void *XL, const void *XR, const void *YL,
                          const void *YR, const void *ZL, const void *ZR, void *R, hipStream_t s)
    {
        if (p == P) return launch_p<T, P>(nb, q, S, XL, XR, YL, YR, ZL, ZR, R, s);
        return Dispatch<T, P - 1>::run(p, nb, q, S, XL, XR, YL, YR, ZL, ZR, R, s);
    }
};
template <typename T>
struct Dispatch<T, 0> {
    static hipError_t run(int, int64_t, int, const void *, const void *, const void *, const void *, const void *,
                          const void *, const void *, void *, hipStream_t)
    {
        return hipErrorInvalidValue;
    }
};

}  // namespace dgr

// Host launcher: 0 on success, a hipError_t otherwise.  p <= 20 (FP64) or
// p <= 24 (FP32) and 1 <= q <= p are checked by the caller.
hipError_t dg_mra_launch(bool fp64, int64_t nb, int p, int q, const void *S, const void *XL, const void *XR,
                         const void *YL, const void *YR, const void *ZL, const void *ZR, void *R, hipStream_t s)
{
    if (nb == 0) return hipSuccess;
    if (fp64) return dgr::Dispatch<double, 20>::run(p, nb, q, S, XL, XR, YL, YR, ZL, ZR, R, s);
    return dgr::Dispatch<float, 24>::run(p, nb, q, S, XL, XR, YL, YR, ZL, ZR, R, s);
}
