// Viscoelastic ADER-DG step (27 quantities: the 9 elastic ones, then 3
// mechanisms x 6 memory variables; Sec. 5.1 names the rheology), FP64.
//   k_visco_predict:  D^{d+1} = sum_dir (Kt_dir D_el) S_dir^T + D^d E^T
//                     (Eq. seissol:derivative with the source term; D_el the
//                     9 elastic columns, the only ones the star matrices S
//                     read), I = sum_d dt^{d+1}/(d+1)! D^d (Eq. seissol:timeint),
//                     face traces R_s^T I_el;
//   k_visco_correct:  Q += sum_dir (Kh_dir I_el) S_dir^T
//                          + sum_s Rh_s [A+_s (R_s^T I_el) + A-_s f^h (R_j^T I_el[nu])]
//                          + I E^T
//                     (Eqs. seissol:correction_local and seissol:correction_neigh
//                     with one lift per face).
// E: stress rows gain -sum_l theta_l, memory rows -omega_l theta_l.
//
// Persistent workgroups of 256 threads walk the elements of a work list (one
// mesh, or the viscoelastic meshes of one degree in a batch).  Every product
// is a chain of v_mfma_f64_16x16x4f64 tiles.  Per element:
//  * predictor: the derivative D^d sits in LDS as [B][27] (basis index as the
//    row); per order one phase computes G_dir = Kt_dir D_el for the three
//    directions and a second phase D^{d+1} = [G_1 G_2 G_3] [S_1 S_2 S_3]^T
//    plus the source, with the time integral accumulated in the registers of
//    the wave that owns each 16 x 16 output tile: two barriers per order;
//  * corrector: phase A computes G_dir = Kh_dir I_el and X_s = f^h x_nbr,
//    phase B the volume product into registers and F_s = [x_own X_s]
//    [A+_s A-_s]^T, phase C adds sum_s Rh_s F_s (one K = 4 Bf product).
// The hierarchical basis makes Kt_dir zero unless the column's degree exceeds
// the row's, and Kh_dir zero unless it is below: the rows of Kt of degree N
// and the columns of Kh of degree N are dropped, and each tile skips the
// k-steps of its zero block.  These reference matrices stay resident in LDS
// for the workgroup's lifetime where two workgroups per CU still fit;
// otherwise the tiles read them from the (L2-resident) blob.
// The workgroup clears its LDS once.  Operand arrays carry zero rows and
// columns up to whole k-steps, and are ordered so that a tile's reads past
// its matrix land in other LDS arrays (or, for the blob, in the next matrix):
// those values only reach output rows or columns that are never stored, so
// the inner loops carry no bounds selects.
// Layouts: Q, I [E][27][B]; star [E][3][27][9]; Aplus, Aminus [E][4][27][9];
// traces [E][4][9][Bf]; the reference blob as dg_reference_matrices writes it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dg_common.h"
#include "visco_internal.h"

// No implicit contraction: every multiply-add below is an explicit fma, so
// all launch shapes (template instantiations) round alike and give the same
// bits.
#pragma clang fp contract(off)

namespace dgv {

using dgk::nb2;
using dgk::nb3;

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int NQ = 27, NE = 9;
constexpr int LDS_TWO_PER_CU = 80 * 1024;

// polynomial degree of basis function r (the basis is ordered by degree)
__host__ __device__ constexpr int deg_of(int r)
{
    int d = 0;
    while (nb3(d) <= r) ++d;
    return d;
}

template <int N, int WVv = (N == 6 ? 8 : 4)>
struct Dim {
    static constexpr int B = nb3(N), Bf = nb2(N), B1 = nb3(N - 1);
    static constexpr int BK = (B + 3) / 4 * 4;             // rows of the derivative arrays (zero beyond B)
    // odd row strides of the LDS matrices read 16 rows at a time (no bank
    // conflicts); B1P also covers whole k-steps (zero columns beyond B1)
    static constexpr int BP = B | 1, B1P = ((B1 + 3) / 4 * 4) | 1, BfP = Bf | 1, WP = 19, TP = 21, PAD = 32;
    static constexpr int MT = (B + 15) / 16, MT1 = (B1 + 15) / 16, MTf = (Bf + 15) / 16;
    // workgroup of WVv waves (by default 4, and 8 at degree 6, whose LDS
    // admits one workgroup per CU; dg_visco_tune may pick the other)
    static constexpr int T = 64 * WVv, WV = WVv, MINW = 2;
    static constexpr int OT = 2 * MT;                      // 16 x 16 tiles of a [B][27] array
    static constexpr int TPW = (OT + WV - 1) / WV;         // of them owned per wave
    static constexpr int QPT = (NQ * B + T - 1) / T;
    // the predictor prefetches the next element into registers below degree 6
    // (at degree 6 the registers go to two waves per SIMD instead)
    static constexpr bool P_PF = N <= 5;
    // predictor LDS (doubles): [Kt rows of degree < N [3][B1][BP] if resident] D, Dn [BK][27], G [B1][27], pad
    static constexpr int P_EL = 2 * BK * NQ + B1 * NQ + PAD, P_KT = 3 * B1 * BP;
    // resident where two workgroups per CU fit; at degree 6 (one wave per
    // SIMD for its registers anyway) resident in the whole LDS
    static constexpr bool P_RES = 8 * (P_EL + P_KT) <= (N == 6 ? 160 * 1024 : LDS_TWO_PER_CU);
    static constexpr int P_LDS = P_EL + (P_RES ? P_KT : 0);
    // corrector LDS: [Kh columns of degree < N [3][B][B1P] if resident] f [3][Bf][BfP], neighbour traces
    // [4][9][Bf], [A+ A-] [4][27][WP], I_el [B][9], G [B][27], [x_own X] [4 Bf][TP], F [4 Bf][27], pad
    static constexpr int C_EL = 3 * Bf * BfP + 4 * NE * Bf + 4 * NQ * WP + B * NE + B * NQ + 4 * Bf * TP +
                                4 * Bf * NQ + PAD;
    static constexpr int C_KH = 3 * B * B1P;
    static constexpr bool C_RES = 8 * (C_EL + C_KH) <= LDS_TWO_PER_CU;
    static constexpr int C_LDS = C_EL + (C_RES ? C_KH : 0);
};

__device__ __forceinline__ d4 mfma(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// a + (E x)[p] for the structured source matrix, x a row of 27 values
__device__ __forceinline__ double add_source(double a, const double *x, int p, double w0, double w1, double w2)
{
    if (p < 6) return a - (x[9 + p] + x[15 + p] + x[21 + p]);
    if (p < 9) return a;
    return fma(-(p < 15 ? w0 : (p < 21 ? w1 : w2)), x[p], a);
}

// the star matrices as the B operand [S_1 S_2 S_3]^T: row k = 9 dir + q,
// column p; the 7 k-steps of column `col` for lane row lk
__device__ __forceinline__ void star_b(const double *Se, int col, int lk, double (&sb)[7])
{
#pragma unroll
    for (int s = 0; s < 7; ++s) {
        const int k = 4 * s + lk, dir = k / NE;
        sb[s] = (k < NQ && col < NQ) ? Se[(dir * NQ + col) * NE + (k - dir * NE)] : 0.0;
    }
}

template <int M>
struct Vals {
    double v[M];
};

// Q + (E I) of the update, for the entries i = tid + u T of an element's [27][B] block
template <int B, int QPT, int T>
__device__ __forceinline__ Vals<QPT> update_operands(const double *Qe, const double *Ig, double w0, double w1,
                                                    double w2, int tid)
{
    Vals<QPT> r;
#pragma unroll
    for (int u = 0; u < QPT; ++u) {
        const int i = tid + u * T, p = i / B, k = i - p * B;
        double v = 0.0;
        if (i < NQ * B) {
            if (p < 6) v = Qe[i] - (Ig[(9 + p) * B + k] + Ig[(15 + p) * B + k] + Ig[(21 + p) * B + k]);
            else if (p < 9) v = Qe[i];
            else v = fma(-(p < 15 ? w0 : (p < 21 ? w1 : w2)), Ig[i], Qe[i]);
        }
        r.v[u] = v;
    }
    return r;
}

// One 16-row tile of G_dir = Kt_dir D_el (rows of degree < N; columns of
// degree <= the tile's lowest row degree are zero and skipped).
template <int N, int MTI, bool RES>
__device__ __forceinline__ d4 kt_tile(const double *Kt_l, const double *Kt_g, const double *Dc, int dir, int li,
                                      int lk)
{
    using Dm = Dim<N>;
    constexpr int B = Dm::B, B1 = Dm::B1, BP = Dm::BP, KS = Dm::BK / 4, KS0 = nb3(deg_of(16 * MTI)) / 4;
    // rows past B1 and columns past 9 are never stored; rows of Dc past B are zero
    const int i = 16 * MTI + li;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = KS0; s < KS; ++s) {
        const int k = 4 * s + lk;
        double a;
        if constexpr (RES) a = Kt_l[(dir * B1 + i) * BP + k];
        else a = Kt_g[(dir * B + i) * B + k];
        acc = mfma(a, Dc[k * NQ + li], acc);
    }
    return acc;
}

// One 16-row tile of G_dir = Kh_dir I_el (columns of degree < N; columns of
// degree >= the tile's highest row degree are zero and skipped).
template <int N, int MTI, bool RES>
__device__ __forceinline__ d4 kh_tile(const double *Kh_l, const double *Kh_g, const double *Iel, int dir, int li,
                                      int lk)
{
    using Dm = Dim<N>;
    constexpr int B = Dm::B, B1 = Dm::B1, B1P = Dm::B1P;
    constexpr int LAST = 16 * MTI + 15 < B - 1 ? 16 * MTI + 15 : B - 1;
    constexpr int KE = (nb3(deg_of(LAST) - 1) + 3) / 4;
    // columns of Kh past B1 are zero (padding in LDS, true zeros in the
    // blob); rows past B and columns past 9 are never stored
    const int i = 16 * MTI + li;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < KE; ++s) {
        const int k = 4 * s + lk;
        double a;
        if constexpr (RES) a = Kh_l[(dir * B + i) * B1P + k];
        else a = Kh_g[(dir * B + i) * B + k];
        acc = mfma(a, Iel[k * NE + li], acc);
    }
    return acc;
}

template <int N, int WVv>
__global__ void __launch_bounds__(64 * WVv) __attribute__((amdgpu_waves_per_eu(2)))
k_visco_predict(const VItem *__restrict__ items, VItem one, int64_t total, const double *__restrict__ blob)
{
    using Dm = Dim<N, WVv>;
    constexpr int B = Dm::B, Bf = Dm::Bf, B1 = Dm::B1, BP = Dm::BP, MT1 = Dm::MT1, MTf = Dm::MTf, OT = Dm::OT,
                  TPW = Dm::TPW, QPT = Dm::QPT;
    constexpr int BK = Dm::BK, KS = BK / 4, THREADS = Dm::T, WAVES = Dm::WV;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    double *const base = reinterpret_cast<double *>(lds_raw);
    double *const Kt_l = base, *const D = base + (Dm::P_RES ? Dm::P_KT : 0), *const Dn = D + BK * NQ,
                 *const G = Dn + BK * NQ;
    const double *Kt_g = blob + 3 * B * B, *R_g = blob + 6 * B * B;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int col = 16 * (wave & 1) + li;    // every tile a wave owns is in column block wave & 1
    for (int i = tid; i < Dm::P_LDS; i += THREADS) base[i] = 0.0;
    __syncthreads();
    if constexpr (Dm::P_RES) {
        for (int i = tid; i < 3 * B1 * B; i += THREADS) {
            const int dr = i / B, k = i - dr * B, dir = dr / B1;
            Kt_l[dr * BP + k] = Kt_g[(dir * B + (dr - dir * B1)) * B + k];
        }
    }
    // below degree 6 the next element's Q and star operands travel in registers
    constexpr int PQ = Dm::P_PF ? QPT : 1;
    double qn[PQ], sn[7];
    VItem it = items ? items[0] : one, nx = it;
    int cur = 0, ncur = 0;
    auto fetch = [&](int64_t gg) {
        while (gg >= nx.first + nx.E) nx = items[++ncur];
        const int64_t ee = gg - nx.first;
        const double *Qe = nx.Q + ee * NQ * B;
#pragma unroll
        for (int u = 0; u < PQ; ++u) {
            const int i = tid + u * THREADS;
            qn[u] = i < NQ * B ? Qe[i] : 0.0;
        }
        star_b(nx.star + ee * 3 * NQ * NE, col, lk, sn);
    };
    if constexpr (Dm::P_PF)
        if ((int64_t)blockIdx.x < total) fetch(blockIdx.x);
    for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
        while (g >= it.first + it.E) it = items[++cur];
        const int64_t e = g - it.first;
        const double dt = it.dt, w0 = it.omega[0], w1 = it.omega[1], w2 = it.omega[2];
        double sb[7];
        __syncthreads();    // the previous element's LDS reads are done (and Kt is staged)
        if constexpr (Dm::P_PF) {
#pragma unroll
            for (int u = 0; u < QPT; ++u) {
                const int i = tid + u * THREADS;
                if (i < NQ * B) {
                    const int p = i / B, k = i - p * B;
                    D[k * NQ + p] = qn[u];
                }
            }
#pragma unroll
            for (int s = 0; s < 7; ++s) sb[s] = sn[s];
            if (g + gridDim.x < total) fetch(g + gridDim.x);
        } else {
            const double *Qe = it.Q + e * NQ * B;
            for (int i = tid; i < NQ * B; i += THREADS) {
                const int p = i / B, k = i - p * B;
                D[k * NQ + p] = Qe[i];
            }
            star_b(it.star + e * 3 * NQ * NE, col, lk, sb);
        }
        __syncthreads();
        d4 Is[TPW];
#pragma unroll
        for (int j = 0; j < TPW; ++j) {
            const int t = wave + WAVES * j, mt = t >> 1;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * mt + lk + 4 * r;
                Is[j][r] = (t < OT && row < B && col < NQ) ? dt * D[row * NQ + col] : 0.0;
            }
        }
        double c = dt;
        double *Dc = D, *Dx = Dn;
        for (int d = 0; d < N; ++d) {
            // G_dir = Kt_dir D_el over the rows of degree < N
            for (int t = wave; t < 3 * MT1; t += WAVES) {
                const int dir = t / MT1, mt = t - dir * MT1;
                d4 acc;
                switch (mt) {
                case 0: acc = kt_tile<N, 0, Dm::P_RES>(Kt_l, Kt_g, Dc, dir, li, lk); break;
                case 1: acc = kt_tile<N, 1, Dm::P_RES>(Kt_l, Kt_g, Dc, dir, li, lk); break;
                case 2: acc = kt_tile<N, 2, Dm::P_RES>(Kt_l, Kt_g, Dc, dir, li, lk); break;
                default: acc = kt_tile<N, 3, Dm::P_RES>(Kt_l, Kt_g, Dc, dir, li, lk); break;
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * mt + lk + 4 * r;
                    if (row < B1 && li < NE) G[row * NQ + dir * NE + li] = acc[r];
                }
            }
            __syncthreads();
            c *= dt / (d + 2);
            // D^{d+1} = [G_1 G_2 G_3] [S_1 S_2 S_3]^T + E D^d;  I += dt^{d+2}/(d+2)! D^{d+1}
#pragma unroll
            for (int j = 0; j < TPW; ++j) {
                const int t = wave + WAVES * j;
                if (t < OT) {
                    const int mt = t >> 1, i = 16 * mt + li;
                    d4 acc = {0.0, 0.0, 0.0, 0.0};
                    if (16 * mt < B1) {
#pragma unroll
                        for (int s = 0; s < 7; ++s) {
                            const int k = 4 * s + lk;
                            acc = mfma((i < B1 && k < NQ) ? G[i * NQ + k] : 0.0, sb[s], acc);
                        }
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = 16 * mt + lk + 4 * r;
                        if (row < B && col < NQ) {
                            const double v = add_source(acc[r], Dc + row * NQ, col, w0, w1, w2);
                            Dx[row * NQ + col] = v;
                            Is[j][r] = fma(c, v, Is[j][r]);
                        }
                    }
                }
            }
            __syncthreads();
            double *tmp = Dc;
            Dc = Dx;
            Dx = tmp;
        }
        // the time integral to LDS (the buffer of the previous derivative), then out
#pragma unroll
        for (int j = 0; j < TPW; ++j) {
            const int t = wave + WAVES * j, mt = t >> 1;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * mt + lk + 4 * r;
                if (t < OT && row < B && col < NQ) Dx[row * NQ + col] = Is[j][r];
            }
        }
        __syncthreads();
        double *Ie = it.I + e * NQ * B;
        for (int i = tid; i < NQ * B; i += THREADS) {
            const int p = i / B, k = i - p * B;
            Ie[i] = Dx[k * NQ + p];
        }
        // face traces R_s^T I_el, stored [s][q][m]
        double *te = it.traces + e * 4 * NE * Bf;
        for (int t = wave; t < 4 * MTf; t += WAVES) {
            const int s = t / MTf, mt = t - s * MTf, i = 16 * mt + li;
            d4 acc = {0.0, 0.0, 0.0, 0.0};
            // rows past Bf read on into the next face's rows (or R-hat) and are
            // never stored; rows of Dx past B are zero
#pragma unroll
            for (int st = 0; st < KS; ++st) {
                const int k = 4 * st + lk;
                acc = mfma(R_g[(s * B + k) * Bf + i], Dx[k * NQ + li], acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = 16 * mt + lk + 4 * r;
                if (m < Bf && li < NE) te[(s * NE + li) * Bf + m] = acc[r];
            }
        }
    }
}

template <int N, int WVv>
__global__ void __launch_bounds__(64 * WVv) __attribute__((amdgpu_waves_per_eu(2)))
k_visco_correct(const VItem *__restrict__ items, VItem one, int64_t total, const double *__restrict__ blob)
{
    using Dm = Dim<N, WVv>;
    constexpr int B = Dm::B, Bf = Dm::Bf, B1 = Dm::B1, B1P = Dm::B1P, BfP = Dm::BfP, WP = Dm::WP, TP = Dm::TP,
                  MT = Dm::MT, MTf = Dm::MTf, OT = Dm::OT, TPW = Dm::TPW;
    constexpr int KSF = (Bf + 3) / 4, KSR = Bf, THREADS = Dm::T, WAVES = Dm::WV, QPT = Dm::QPT;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    double *const base = reinterpret_cast<double *>(lds_raw);
    double *const Kh_l = base, *const f_l = base + (Dm::C_RES ? Dm::C_KH : 0), *const Tn = f_l + 3 * Bf * BfP,
                 *const W = Tn + 4 * NE * Bf, *const Iel = W + 4 * NQ * WP, *const G = Iel + B * NE,
                 *const T = G + B * NQ, *const F = T + 4 * Bf * TP;
    const double *Kh_g = blob, *Rh_g = blob + 6 * B * B + 4 * B * Bf, *f_g = Rh_g + 4 * B * Bf;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, li = lane & 15, lk = lane >> 4;
    const int col = 16 * (wave & 1) + li;    // every owned output tile is in column block wave & 1
    for (int i = tid; i < Dm::C_LDS; i += THREADS) base[i] = 0.0;
    __syncthreads();
    for (int i = tid; i < 3 * Bf * Bf; i += THREADS) {
        const int r = i / Bf;
        f_l[r * BfP + (i - r * Bf)] = f_g[i];
    }
    if constexpr (Dm::C_RES) {
        for (int i = tid; i < 3 * B * B1; i += THREADS) {
            const int dr = i / B1;
            Kh_l[dr * B1P + (i - dr * B1)] = Kh_g[dr * B + (i - dr * B1)];
        }
    }
    // The element's inputs: elastic columns of I, own traces, neighbour
    // traces (gathered), A+ and A-; at degrees 2, 3 and 5 those of the next
    // element are fetched into registers while this one computes (at degree 4
    // the registers would spill at two waves per SIMD, at degree 6 they go to
    // the eight waves of the workgroup).
    constexpr bool PF = N <= 5 && N != 4;
    constexpr int PI = PF ? (NE * B + THREADS - 1) / THREADS : 1, PT = PF ? (4 * NE * Bf + THREADS - 1) / THREADS : 1,
                  PA = PF ? (4 * NQ * NE + THREADS - 1) / THREADS : 1;
    double ri[PI], rto[PT], rtn[PT], rap[PA], ram[PA], sn[7];
    VItem it = items ? items[0] : one, nx = it;
    int cur = 0, ncur = 0;
    auto fetch = [&](int64_t gg) {
        while (gg >= nx.first + nx.E) nx = items[++ncur];
        const int64_t ee = gg - nx.first;
        const double *Ig = nx.I + ee * NQ * B, *to = nx.traces + ee * 4 * NE * Bf;
        const double *ap = nx.Ap + ee * 4 * NQ * NE, *am = nx.Am + ee * 4 * NQ * NE;
#pragma unroll
        for (int u = 0; u < PI; ++u) {
            const int i = tid + u * THREADS;
            ri[u] = i < NE * B ? Ig[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < PT; ++u) {
            const int i = tid + u * THREADS;
            rto[u] = i < 4 * NE * Bf ? to[i] : 0.0;
            double v = 0.0;
            if (i < 4 * NE * Bf) {
                const int s = i / (NE * Bf), r = i - s * NE * Bf;
                const int32_t nu = nx.neigh[ee * 4 + s];
                if (nu >= 0 && nu < nx.E)
                    v = nx.traces[((int64_t)nu * 4 + (nx.face_rot[ee * 4 + s] & 3)) * NE * Bf + r];
            }
            rtn[u] = v;
        }
#pragma unroll
        for (int u = 0; u < PA; ++u) {
            const int i = tid + u * THREADS;
            rap[u] = i < 4 * NQ * NE ? ap[i] : 0.0;
            ram[u] = i < 4 * NQ * NE ? am[i] : 0.0;
        }
        star_b(nx.star + ee * 3 * NQ * NE, col, lk, sn);
    };
    if constexpr (PF)
        if ((int64_t)blockIdx.x < total) fetch(blockIdx.x);
    for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
        while (g >= it.first + it.E) it = items[++cur];
        const int64_t e = g - it.first;
        const double *Ig = it.I + e * NQ * B;
        double sb[7];
        __syncthreads();    // the previous element's LDS reads are done (and f, Kh are staged)
        if constexpr (PF) {
#pragma unroll
            for (int u = 0; u < PI; ++u) {
                const int i = tid + u * THREADS;
                if (i < NE * B) {
                    const int p = i / B, k = i - p * B;
                    Iel[k * NE + p] = ri[u];
                }
            }
#pragma unroll
            for (int u = 0; u < PT; ++u) {
                const int i = tid + u * THREADS;
                if (i < 4 * NE * Bf) {
                    const int s = i / (NE * Bf), r = i - s * NE * Bf, q = r / Bf, m = r - q * Bf;
                    T[(s * Bf + m) * TP + q] = rto[u];
                    Tn[i] = rtn[u];
                }
            }
#pragma unroll
            for (int u = 0; u < PA; ++u) {
                const int i = tid + u * THREADS;
                if (i < 4 * NQ * NE) {
                    const int sp = i / NE, q = i - sp * NE;
                    W[sp * WP + q] = rap[u];
                    W[sp * WP + NE + q] = ram[u];
                }
            }
#pragma unroll
            for (int s = 0; s < 7; ++s) sb[s] = sn[s];
            if (g + gridDim.x < total) fetch(g + gridDim.x);
        } else {
            star_b(it.star + e * 3 * NQ * NE, col, lk, sb);
            for (int i = tid; i < NE * B; i += THREADS) {
                const int p = i / B, k = i - p * B;
                Iel[k * NE + p] = Ig[i];
            }
            const double *to = it.traces + e * 4 * NE * Bf;
            for (int i = tid; i < 4 * NE * Bf; i += THREADS) {
                const int s = i / (NE * Bf), r = i - s * NE * Bf, q = r / Bf, m = r - q * Bf;
                T[(s * Bf + m) * TP + q] = to[i];
                const int32_t nu = it.neigh[e * 4 + s];
                double v = 0.0;
                if (nu >= 0 && nu < it.E)
                    v = it.traces[((int64_t)nu * 4 + (it.face_rot[e * 4 + s] & 3)) * NE * Bf + r];
                Tn[i] = v;
            }
            const double *ap = it.Ap + e * 4 * NQ * NE, *am = it.Am + e * 4 * NQ * NE;
            for (int i = tid; i < 4 * NQ * NE; i += THREADS) {
                const int sp = i / NE, q = i - sp * NE;
                W[sp * WP + q] = ap[i];
                W[sp * WP + NE + q] = am[i];
            }
        }
        // the update's Q and source term E I: loaded before phase A where the
        // next element is prefetched (the latency hides behind phases A to C;
        // at degrees 4 and 6 the longer live range costs more than it hides),
        // else before phase B; used after phase C
        double *const Qe = it.Q + e * NQ * B;
        const double w0 = it.omega[0], w1 = it.omega[1], w2 = it.omega[2];
        Vals<QPT> qv;
        if constexpr (PF) qv = update_operands<B, QPT, THREADS>(Qe, Ig, w0, w1, w2, tid);
        __syncthreads();
        // phase A: G_dir = Kh_dir I_el (columns of degree < N);  X_s = f^h x_nbr
        for (int t = wave; t < 3 * MT + 4 * MTf; t += WAVES) {
            if (t < 3 * MT) {
                const int dir = t / MT, mt = t - dir * MT;
                d4 acc;
                switch (mt) {
                case 0: acc = kh_tile<N, 0, Dm::C_RES>(Kh_l, Kh_g, Iel, dir, li, lk); break;
                case 1: acc = kh_tile<N, 1, Dm::C_RES>(Kh_l, Kh_g, Iel, dir, li, lk); break;
                case 2: acc = kh_tile<N, 2, Dm::C_RES>(Kh_l, Kh_g, Iel, dir, li, lk); break;
                case 3: acc = kh_tile<N, 3, Dm::C_RES>(Kh_l, Kh_g, Iel, dir, li, lk); break;
                case 4: acc = kh_tile<N, 4, Dm::C_RES>(Kh_l, Kh_g, Iel, dir, li, lk); break;
                default: acc = kh_tile<N, 5, Dm::C_RES>(Kh_l, Kh_g, Iel, dir, li, lk); break;
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * mt + lk + 4 * r;
                    if (row < B && li < NE) G[row * NQ + dir * NE + li] = acc[r];
                }
            } else {
                const int tt = t - 3 * MT, s = tt / MTf, mt = tt - s * MTf, i = 16 * mt + li;
                // orientations above 2 are invalid input; they read f^0 so
                // that the read stays inside the matrix
                const int h0 = (it.face_rot[e * 4 + s] >> 2) & 3, h = h0 > 2 ? 0 : h0;
                d4 acc = {0.0, 0.0, 0.0, 0.0};
                // rows past Bf and columns past 9 are never stored; the k-step
                // past Bf meets the zero of the select
#pragma unroll
                for (int st = 0; st < KSF; ++st) {
                    const int k = 4 * st + lk;
                    acc = mfma(f_l[(h * Bf + i) * BfP + k], k < Bf ? Tn[(s * NE + li) * Bf + k] : 0.0, acc);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * mt + lk + 4 * r;
                    if (row < Bf && li < NE) T[(s * Bf + row) * TP + NE + li] = acc[r];
                }
            }
        }
        __syncthreads();
        if constexpr (!PF) qv = update_operands<B, QPT, THREADS>(Qe, Ig, w0, w1, w2, tid);
        // phase B: volume [G_1 G_2 G_3] [S_1 S_2 S_3]^T into the owned tiles;
        // F_s = [x_own X_s] [A+_s A-_s]^T
        d4 acc[TPW];
#pragma unroll
        for (int j = 0; j < TPW; ++j) {
            const int t = wave + WAVES * j, i = 16 * (t >> 1) + li;
            acc[j] = d4{0.0, 0.0, 0.0, 0.0};
            if (t < OT) {
#pragma unroll
                for (int s = 0; s < 7; ++s) {
                    const int k = 4 * s + lk;
                    acc[j] = mfma(G[i * NQ + k], sb[s], acc[j]);   // rows past B never stored; sb is 0 past k = 26
                }
            }
        }
        for (int t = wave; t < 8 * MTf; t += WAVES) {
            const int s = t / (2 * MTf), r2 = t - s * 2 * MTf, mt = r2 >> 1;
            const int i = 16 * mt + li, fc = 16 * (r2 & 1) + li;
            d4 f = {0.0, 0.0, 0.0, 0.0};
            // columns 18-20 of T are zero; rows past Bf and columns past 27 are never stored
#pragma unroll
            for (int st = 0; st < 5; ++st) {
                const int k = 4 * st + lk;
                f = mfma(T[(s * Bf + i) * TP + k], W[(s * NQ + fc) * WP + k], f);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * mt + lk + 4 * r;
                if (row < Bf && fc < NQ) F[(s * Bf + row) * NQ + fc] = f[r];
            }
        }
        __syncthreads();
        // phase C: + sum_s Rh_s F_s as one product over K = 4 Bf; the result
        // to LDS (G is free after phase B)
#pragma unroll
        for (int j = 0; j < TPW; ++j) {
            const int t = wave + WAVES * j, mt = t >> 1, i = 16 * mt + li;
            if (t < OT) {
                // chunks of 7 k-steps keep the loads in flight (and the registers) bounded
#pragma unroll 7
                for (int st = 0; st < KSR; ++st) {
                    const int kk = 4 * st + lk, s = kk / Bf, m = kk - s * Bf;
                    // rows past B read on into the next face's rows (or f) and are never stored
                    acc[j] = mfma(Rh_g[(s * B + i) * Bf + m], F[kk * NQ + col], acc[j]);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = 16 * mt + lk + 4 * r;
                    if (row < B && col < NQ) G[row * NQ + col] = acc[j][r];
                }
            }
        }
        __syncthreads();
        // Q += volume + fluxes + E I
#pragma unroll
        for (int u = 0; u < QPT; ++u) {
            const int i = tid + u * THREADS, p = i / B, k = i - p * B;
            if (i < NQ * B) Qe[i] = qv.v[u] + G[k * NQ + p];
        }
    }
}

template <typename K>
hipError_t occupancy(K kernel, int threads, size_t lds, int *per_cu)
{
    hipError_t e = hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, (const void *)kernel, threads, lds);
    if (e == hipSuccess && *per_cu < 1) *per_cu = 1;
    return e;
}

template <int N, int WVv>
struct Occ {
    static inline int cus = 0, predict = 0, correct = 0;    // CUs and resident workgroups per CU, set once
};

template <int N, int WVv>
hipError_t prepare()
{
    using Dm = Dim<N, WVv>;
    using O = Occ<N, WVv>;
    if (O::cus) return hipSuccess;
    int dev = 0, cus = 0, a = 0, b = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = occupancy(k_visco_predict<N, WVv>, Dm::T, (size_t)Dm::P_LDS * 8, &a);
    if (e == hipSuccess) e = occupancy(k_visco_correct<N, WVv>, Dm::T, (size_t)Dm::C_LDS * 8, &b);
    if (e != hipSuccess) return e;
    O::predict = a, O::correct = b, O::cus = cus;
    return hipSuccess;
}

// One step over the work list: persistent grids of CUs x min(per_cu, the
// resident limit) workgroups (per_cu 0: the resident limit).
template <int N, int WVv>
hipError_t step(const VItem *items, const VItem &one, int64_t total, const double *blob, int per_cu, hipStream_t s)
{
    using Dm = Dim<N, WVv>;
    using O = Occ<N, WVv>;
    hipError_t e = prepare<N, WVv>();
    if (e != hipSuccess) return e;
    const int64_t gp = (int64_t)O::cus * (per_cu > 0 && per_cu < O::predict ? per_cu : O::predict);
    const int64_t gc = (int64_t)O::cus * (per_cu > 0 && per_cu < O::correct ? per_cu : O::correct);
    const unsigned np = (unsigned)(total < gp ? total : gp), nc = (unsigned)(total < gc ? total : gc);
    hipLaunchKernelGGL((k_visco_predict<N, WVv>), dim3(np), dim3(Dm::T), (size_t)Dm::P_LDS * 8, s, items, one,
                       total, blob);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_visco_correct<N, WVv>), dim3(nc), dim3(Dm::T), (size_t)Dm::C_LDS * 8, s, items, one,
                       total, blob);
    return hipGetLastError();
}

template <int N>
hipError_t step_shape(int waves, const VItem *items, const VItem &one, int64_t total, const double *blob,
                      int per_cu, hipStream_t s)
{
    return waves == 8 ? step<N, 8>(items, one, total, blob, per_cu, s) : step<N, 4>(items, one, total, blob, per_cu, s);
}

template <int N>
hipError_t prepare_shape(int waves, int *max_per_cu)
{
    hipError_t e = waves == 8 ? prepare<N, 8>() : prepare<N, 4>();
    if (e == hipSuccess && max_per_cu)
        *max_per_cu = waves == 8 ? (Occ<N, 8>::predict > Occ<N, 8>::correct ? Occ<N, 8>::predict : Occ<N, 8>::correct)
                                 : (Occ<N, 4>::predict > Occ<N, 4>::correct ? Occ<N, 4>::predict : Occ<N, 4>::correct);
    return e;
}

// the launch shape of each degree (process-wide): waves per workgroup, resident workgroups per CU (0: all that fit)
VShape g_shape[7] = {{4, 0}, {4, 0}, {4, 0}, {4, 0}, {4, 0}, {4, 0}, {8, 0}};

}  // namespace dgv

VShape visco_shape(int degree) { return degree >= 2 && degree <= 6 ? dgv::g_shape[degree] : VShape{4, 0}; }

void visco_set_shape(int degree, VShape shape)
{
    if (degree >= 2 && degree <= 6) dgv::g_shape[degree] = shape;
}

hipError_t visco_prepare_shape(int degree, int waves, int *max_per_cu)
{
    switch (degree) {
    case 2: return dgv::prepare_shape<2>(waves, max_per_cu);
    case 3: return dgv::prepare_shape<3>(waves, max_per_cu);
    case 4: return dgv::prepare_shape<4>(waves, max_per_cu);
    case 5: return dgv::prepare_shape<5>(waves, max_per_cu);
    case 6: return dgv::prepare_shape<6>(waves, max_per_cu);
    default: return hipErrorInvalidValue;
    }
}

hipError_t visco_prepare(int degree) { return visco_prepare_shape(degree, visco_shape(degree).waves, nullptr); }

hipError_t visco_step_shape(int degree, VShape shape, const VItem *items, int n_items, const VItem &one,
                            int64_t total, const double *blob, hipStream_t s)
{
    if (total <= 0 || n_items <= 0) return hipSuccess;
    switch (degree) {
    case 2: return dgv::step_shape<2>(shape.waves, items, one, total, blob, shape.per_cu, s);
    case 3: return dgv::step_shape<3>(shape.waves, items, one, total, blob, shape.per_cu, s);
    case 4: return dgv::step_shape<4>(shape.waves, items, one, total, blob, shape.per_cu, s);
    case 5: return dgv::step_shape<5>(shape.waves, items, one, total, blob, shape.per_cu, s);
    case 6: return dgv::step_shape<6>(shape.waves, items, one, total, blob, shape.per_cu, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t visco_step_launch(int degree, const VItem *items, int n_items, const VItem &one, int64_t total,
                             const double *blob, hipStream_t s)
{
    return visco_step_shape(degree, visco_shape(degree), items, n_items, one, total, blob, s);
}
