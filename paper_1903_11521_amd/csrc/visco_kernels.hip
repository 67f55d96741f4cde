// Viscoelastic ADER-DG step (27 quantities: the 9 elastic ones, then 3
// mechanisms x 6 memory variables; Sec. 5.1 names the rheology).  Per
// element, FP64, one workgroup of 256 threads:
//   k_visco_predict:  D^{d+1} = sum_dir (Kt_dir D_el^T) S_dir^T + D^d E^T
//                     (Eq. seissol:derivative with the source term; D_el the
//                     9 elastic columns, the only ones the star matrices S
//                     read), I = sum_d dt^{d+1}/(d+1)! D^d (Eq. seissol:timeint),
//                     face traces R_s^T I_el;
//   k_visco_correct:  Q += sum_dir (Kh_dir I_el^T) S_dir^T
//                          + sum_s Rh_s [A+_s (R_s^T I_el) + A-_s f^h (R_j^T I_el[nu])]
//                          + I E^T
//                     (Eqs. seissol:correction_local and seissol:correction_neigh
//                     with one lift per face).
// E: stress rows gain -sum_l theta_l, memory rows -omega_l theta_l.
// The element's arrays live in LDS with the basis index as the row
// ([B][27]); every reference-matrix product is a small GEMM on the matrix
// cores (v_mfma_f64_16x16x4f64) with the reference matrix staged in LDS.
// Layouts: Q, I [E][27][B]; star [E][3][27][9]; Aplus, Aminus [E][4][27][9];
// traces [E][4][9][Bf]; the reference blob as dg_reference_matrices writes it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dg_common.h"
#include "visco_internal.h"

namespace dgv {

using dgk::nb2;
using dgk::nb3;

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int NQ = 27, NE = 9, THREADS = 256, WAVES = THREADS / 64;

// C (+)= A B (M x K times K x N), operands at A[i ar + k ac], B[k br + j bc],
// C[i cr + j cc].  16 x 16 tiles dealt to the waves; MFMA lane layout: A[i][k]
// in lane 16k + i, B[k][j] in lane 16k + j, output register r of lane l is
// row l/16 + 4r, column l%16.  The caller synchronises around it.
__device__ void gemm(int M, int N, int K, const double *A, int ar, int ac, const double *B, int br, int bc,
                     double *C, int cr, int cc, bool acc)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int MT = (M + 15) >> 4, NT = (N + 15) >> 4, KS = (K + 3) >> 2;
    for (int t = wave; t < MT * NT; t += WAVES) {
        const int mt = t / NT, nt = t - mt * NT;
        const int i = 16 * mt + li, j = 16 * nt + li;
        d4 c = {0.0, 0.0, 0.0, 0.0};
        for (int s = 0; s < KS; ++s) {
            const int k = 4 * s + lk;
            const double a = (i < M && k < K) ? A[i * ar + k * ac] : 0.0;
            const double b = (k < K && j < N) ? B[k * br + j * bc] : 0.0;
            c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * mt + lk + 4 * r;
            if (row < M && j < N) {
                double *o = C + row * cr + j * cc;
                *o = acc ? *o + c[r] : c[r];
            }
        }
    }
}

__device__ __forceinline__ void copy(double *dst, const double *__restrict__ src, int n)
{
    for (int i = threadIdx.x; i < n; i += THREADS) dst[i] = src[i];
}

// (E x)[p] for the structured source matrix, x a row of 27 values
__device__ __forceinline__ double source(const double *x, int p, const double *omega)
{
    if (p < 6) return -(x[9 + p] + x[15 + p] + x[21 + p]);
    if (p < 9) return 0.0;
    return -omega[(p - 9) / 6] * x[p];
}

struct Ref {
    const double *Kh, *Kt, *R, *Rh, *f;
};

template <int N>
__device__ __forceinline__ Ref ref_of(const double *blob)
{
    constexpr int B = nb3(N), Bf = nb2(N);
    Ref r;
    r.Kh = blob;
    r.Kt = blob + 3 * B * B;
    r.R = blob + 6 * B * B;
    r.Rh = r.R + 4 * B * Bf;
    r.f = r.Rh + 4 * B * Bf;
    return r;
}

template <int N>
constexpr int predict_lds() { return 3 * nb3(N) * NQ + nb3(N) * nb3(N) + NE * nb3(N) + 3 * NQ * NE + NE * nb2(N); }
template <int N>
constexpr int correct_lds() { return 2 * nb3(N) * NQ + nb3(N) * nb3(N) + NE * nb3(N) + 3 * NQ * NE + 3 * NE * nb2(N) + NQ * nb2(N); }

template <int N>
__global__ void __launch_bounds__(THREADS)
k_visco_predict(double dt, const double *__restrict__ Q, const double *__restrict__ star, VOmega om,
                const double *__restrict__ blob, double *__restrict__ Iout, double *__restrict__ traces)
{
    constexpr int B = nb3(N), Bf = nb2(N);
    extern __shared__ __align__(16) unsigned char lds_raw[];
    double *D = reinterpret_cast<double *>(lds_raw), *Dn = D + B * NQ, *Is = Dn + B * NQ, *Mb = Is + B * NQ,
           *G = Mb + B * B, *S = G + NE * B, *tr = S + 3 * NQ * NE;
    const Ref rf = ref_of<N>(blob);
    const int64_t e = blockIdx.x;
    const double *Qe = Q + e * NQ * B;
    for (int i = threadIdx.x; i < NQ * B; i += THREADS) {
        const int p = i / B, k = i - p * B;
        const double v = Qe[i];
        D[k * NQ + p] = v;
        Is[k * NQ + p] = dt * v;
    }
    copy(S, star + e * 3 * NQ * NE, 3 * NQ * NE);
    double c = dt;
    for (int d = 0; d < N; ++d) {
        for (int dir = 0; dir < 3; ++dir) {
            __syncthreads();
            copy(Mb, rf.Kt + dir * B * B, B * B);
            __syncthreads();
            gemm(B, NE, B, Mb, B, 1, D, NQ, 1, G, NE, 1, false);                      // G = Kt D_el^T
            __syncthreads();
            gemm(B, NQ, NE, G, NE, 1, S + dir * NQ * NE, 1, NE, Dn, NQ, 1, dir > 0);  // Dn (+)= G S^T
        }
        __syncthreads();
        c *= dt / (d + 2);
        for (int i = threadIdx.x; i < NQ * B; i += THREADS) {
            const int k = i / NQ, p = i - k * NQ;
            const double v = Dn[i] + source(D + k * NQ, p, om.w);
            Dn[i] = v;
            Is[i] += c * v;
        }
        __syncthreads();
        double *t = D;
        D = Dn;
        Dn = t;
    }
    double *Ie = Iout + e * NQ * B;
    for (int i = threadIdx.x; i < NQ * B; i += THREADS) {
        const int p = i / B, k = i - p * B;
        Ie[i] = Is[k * NQ + p];
    }
    for (int s = 0; s < 4; ++s) {
        __syncthreads();
        copy(Mb, rf.R + s * B * Bf, B * Bf);
        __syncthreads();
        gemm(Bf, NE, B, Mb, 1, Bf, Is, NQ, 1, tr, NE, 1, false);                     // tr = R_s^T I_el
        __syncthreads();
        double *te = traces + (e * 4 + s) * NE * Bf;
        for (int i = threadIdx.x; i < NE * Bf; i += THREADS) {
            const int q = i / Bf, m = i - q * Bf;
            te[i] = tr[m * NE + q];
        }
    }
}

template <int N>
__global__ void __launch_bounds__(THREADS)
k_visco_correct(int64_t E, const double *__restrict__ I, const double *__restrict__ traces,
                const double *__restrict__ star, const double *__restrict__ Ap, const double *__restrict__ Am,
                const int32_t *__restrict__ neigh, const uint8_t *__restrict__ face_rot, VOmega om,
                const double *__restrict__ blob, double *__restrict__ Q)
{
    constexpr int B = nb3(N), Bf = nb2(N);
    extern __shared__ __align__(16) unsigned char lds_raw[];
    double *Is = reinterpret_cast<double *>(lds_raw), *acc = Is + B * NQ, *Mb = acc + B * NQ, *G = Mb + B * B,
           *S = G + NE * B, *trO = S + 3 * NQ * NE, *trN = trO + NE * Bf, *X = trN + NE * Bf, *F = X + NE * Bf;
    const Ref rf = ref_of<N>(blob);
    const int64_t e = blockIdx.x;
    const double *Ie = I + e * NQ * B;
    for (int i = threadIdx.x; i < NQ * B; i += THREADS) {
        const int p = i / B, k = i - p * B;
        Is[k * NQ + p] = Ie[i];
    }
    copy(S, star + e * 3 * NQ * NE, 3 * NQ * NE);
    // volume
    for (int dir = 0; dir < 3; ++dir) {
        __syncthreads();
        copy(Mb, rf.Kh + dir * B * B, B * B);
        __syncthreads();
        gemm(B, NE, B, Mb, B, 1, Is, NQ, 1, G, NE, 1, false);                        // G = Kh I_el^T
        __syncthreads();
        gemm(B, NQ, NE, G, NE, 1, S + dir * NQ * NE, 1, NE, acc, NQ, 1, dir > 0);   // acc (+)= G S^T
    }
    // faces: one lift of A+ x_own + A- f^h x_nbr per face
    for (int s = 0; s < 4; ++s) {
        const int32_t nu = neigh[e * 4 + s];
        const bool has = nu >= 0 && nu < E;
        // orientations above 2 are invalid input; they read f^0 so that the
        // read stays inside the blob
        const int j = face_rot[e * 4 + s] & 3, h0 = (face_rot[e * 4 + s] >> 2) & 3, h = h0 > 2 ? 0 : h0;
        __syncthreads();
        const double *to = traces + (e * 4 + s) * NE * Bf;
        for (int i = threadIdx.x; i < NE * Bf; i += THREADS) {
            const int q = i / Bf, m = i - q * Bf;
            trO[m * NE + q] = to[i];
        }
        if (has) {
            const double *tn = traces + ((int64_t)nu * 4 + j) * NE * Bf;
            for (int i = threadIdx.x; i < NE * Bf; i += THREADS) {
                const int q = i / Bf, m = i - q * Bf;
                trN[m * NE + q] = tn[i];
            }
            copy(Mb, rf.f + h * Bf * Bf, Bf * Bf);
            __syncthreads();
            gemm(Bf, NE, Bf, Mb, Bf, 1, trN, NE, 1, X, NE, 1, false);                // X = f^h x_nbr
        } else {
            for (int i = threadIdx.x; i < NE * Bf; i += THREADS) X[i] = 0.0;
        }
        __syncthreads();
        const double *ap = Ap + (e * 4 + s) * NQ * NE, *am = Am + (e * 4 + s) * NQ * NE;
        for (int i = threadIdx.x; i < Bf * NQ; i += THREADS) {
            const int m = i / NQ, p = i - m * NQ;
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < NE; ++q) v = fma(ap[p * NE + q], trO[m * NE + q], fma(am[p * NE + q], X[m * NE + q], v));
            F[i] = v;
        }
        copy(Mb, rf.Rh + s * B * Bf, B * Bf);
        __syncthreads();
        gemm(B, NQ, Bf, Mb, Bf, 1, F, NQ, 1, acc, NQ, 1, true);                      // acc += Rh_s F
    }
    __syncthreads();
    double *Qe = Q + e * NQ * B;
    for (int i = threadIdx.x; i < NQ * B; i += THREADS) {
        const int p = i / B, k = i - p * B;
        Qe[i] += acc[k * NQ + p] + source(Is + k * NQ, p, om.w);
    }
}

template <int N>
hipError_t step(int64_t E, double dt, double *Q, double *I, double *traces, const double *star, const double *Ap,
                const double *Am, const int32_t *neigh, const uint8_t *face_rot, VOmega om, const double *blob,
                hipStream_t s)
{
    static bool attr = false;      // the dynamic LDS limits, set once per degree
    const size_t lp = (size_t)predict_lds<N>() * 8, lc = (size_t)correct_lds<N>() * 8;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_visco_predict<N>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lp);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)k_visco_correct<N>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lc);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_visco_predict<N>, dim3((unsigned)E), dim3(THREADS), lp, s, dt, Q, star, om, blob, I,
                       traces);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_visco_correct<N>, dim3((unsigned)E), dim3(THREADS), lc, s, E, I, traces, star, Ap, Am,
                       neigh, face_rot, om, blob, Q);
    return hipGetLastError();
}

}  // namespace dgv

hipError_t visco_step_launch(int degree, int64_t E, double dt, double *Q, double *I, double *traces,
                             const double *star, const double *Ap, const double *Am, const int32_t *neigh,
                             const uint8_t *face_rot, VOmega om, const double *blob, hipStream_t s)
{
    switch (degree) {
    case 2: return dgv::step<2>(E, dt, Q, I, traces, star, Ap, Am, neigh, face_rot, om, blob, s);
    case 3: return dgv::step<3>(E, dt, Q, I, traces, star, Ap, Am, neigh, face_rot, om, blob, s);
    case 4: return dgv::step<4>(E, dt, Q, I, traces, star, Ap, Am, neigh, face_rot, om, blob, s);
    case 5: return dgv::step<5>(E, dt, Q, I, traces, star, Ap, Am, neigh, face_rot, om, blob, s);
    case 6: return dgv::step<6>(E, dt, Q, I, traces, star, Ap, Am, neigh, face_rot, om, blob, s);
    default: return hipErrorInvalidValue;
    }
}
