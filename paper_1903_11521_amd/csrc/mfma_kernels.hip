// Split-BF16 matrix-core form of the step kernels (Sec. 5.1.1, Eqs.
// seissol:derivative, seissol:timeint, seissol:correction_local,
// seissol:correction_neigh), for CDNA4 (gfx950).
//
// Every reference-matrix contraction (K-tilde, K-hat, R^T, R-hat, f^h) is a
// GEMM whose A operand is the element-independent matrix and whose B operand
// is one quantity column of 16 elements: v_mfma_f32_16x16x32_bf16 with three
// products, A_hi B_hi + A_hi B_lo + A_lo B_hi (x_hi = bf16(x),
// x_lo = bf16(x - x_hi), round to nearest even), accumulated in FP32.  The
// dropped A_lo B_lo term and the two representation errors bound one product's
// relative error by about 3 * 2^-16.  The star matrices (sparse, per element)
// and the flux solvers A+/A- (dense 9 x 9 per face, FP64) mix the quantity
// columns of one element, which a lane holds entirely (all 9 columns of its
// element, its rows), so those products are lane-local VALU work; A+/A- run in
// FP64 on FP32 traces and are rounded once.
//
// Two tilings share the code (Tile<FUSED>): a wave takes 16 elements, one per
// MFMA column, or (fused simulations, the extra index s of Q_kps in Sec.
// 5.1.1) one element and 16 simulations of it, one per column; then the
// star matrices, flux solvers and neighbour relations are the same for the
// whole wave.
//
// Lane layout (one 64-lane wave): lane = 16 G + c, c the MFMA column; the
// lane holds, for every quantity column of its element (and simulation) and
// every 16-row tile m, the basis rows 16 m + 4 G + r (r = 0..3), an f32x4.  That is
// where an MFMA leaves output tile m, and in K step s a lane feeds its rows of
// tiles 2 s and 2 s + 1 as the eight K values 8 G .. 8 G + 7 (the fragment
// tables are generated for this order), so a chain of contractions never
// moves data between lanes.  Rows past a column's end are zero in registers
// and never stored.
#include "dg_common.h"
#include "mfma_tables.h"

namespace dgm {

using dgk::nb2;
using dgk::nb3;
using dgk::static_for;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int EPT = 16;                 // elements per wave (MFMA N dimension)
constexpr int NQ = 9;

__host__ __device__ constexpr int tiles(int rows) { return (rows + 15) / 16; }
__host__ __device__ constexpr int ksteps(int rows) { return (rows + 31) / 32; }

// Coupling columns of the packed star row p (slot 2 of rows 3..5 is padding
// with a zero coefficient; it repeats slot 0's column).
__host__ __device__ constexpr int star_q(int p, int slot)
{
    constexpr int t[9][3] = {{6, 7, 8}, {6, 7, 8}, {6, 7, 8}, {6, 7, 6}, {7, 8, 7},
                             {6, 8, 6}, {0, 3, 5}, {1, 3, 4}, {2, 4, 5}};
    return t[p][slot];
}

// Addressing of a wave's 16 MFMA columns.
//   FUSED = false: 16 consecutive elements (column c = element base + c);
//     DOF arrays [E][9][R], traces [E][4][9][Bf], rows contiguous.
//   FUSED = true:  one element (the workgroup's), 16 simulations (column c =
//     simulation c); DOF arrays [E][9][R][16], traces [E][4][9][Bf][16]:
//     a row of one quantity holds the 16 simulations side by side.
// Per-element data (star, flux solvers, neighbours) is staged per element
// slot: 16 slots, or 1.
template <bool FUSED>
struct Tile {
    static constexpr int RS = FUSED ? EPT : 1;      // row stride of a DOF column
    static constexpr int SLOTS = FUSED ? 1 : EPT;   // elements per wave
    int lane, c, G;
    int64_t base;   // first element of the wave
    int64_t elem;   // this lane's element, clamped into [0, E)
    int slot;       // its element slot
    bool active;    // its element is < E
    int64_t nvalid; // elements of the wave below E

    __device__ __forceinline__ Tile(int64_t E, int64_t lb)
    {
        lane = threadIdx.x;
        c = lane & 15;
        G = lane >> 4;
        if constexpr (FUSED) {
            base = lb;
            elem = lb;
            slot = 0;
            active = true;
            nvalid = 1;
        } else {
            base = lb * EPT;
            const int64_t el = base + c;
            active = el < E;
            elem = el < E ? el : E - 1;
            slot = c;
            nvalid = (E - base) < EPT ? (E - base) : EPT;
        }
    }
    // column q of element el in an array of R rows per quantity
    template <int R, typename T>
    __device__ __forceinline__ T *col(T *X, int64_t el, int q) const
    {
        if constexpr (FUSED) return X + (el * NQ + q) * R * EPT + c;
        else return X + (el * NQ + q) * R;
    }
    // column q of face s of element el in a trace array
    template <int Bf, typename T>
    __device__ __forceinline__ T *tcol(T *tr, int64_t el, int s, int q) const
    {
        if constexpr (FUSED) return tr + ((el * 4 + s) * NQ + q) * Bf * EPT + c;
        else return tr + ((el * 4 + s) * NQ + q) * Bf;
    }
};

__device__ __forceinline__ f32x4 zero4() { return f32x4{0.f, 0.f, 0.f, 0.f}; }

// Rows 16 m + 4 G .. +3 of a column of R rows starting at `col`, rows RS
// values apart (dword-aligned), zero past the end.  RS = 1: the four values
// are contiguous; in a partial tile every lane loads four in-range rows
// ending at row R - 1 at the latest and moves its own rows into place with
// selects, so there is no divergent branch around the load.  RS > 1: four
// loads, each from an in-range row, selected to zero past the end.
template <int R, int RS = 1>
__device__ __forceinline__ f32x4 load_tile(const float *col, int m, int G)
{
    static_assert(R >= 4, "columns have at least 4 rows");
    const int r0 = 16 * m + 4 * G;
    if constexpr (RS > 1) {
        f32x4 v;
        if (16 * m + 16 <= R) {
            const float *c = col + r0 * RS;
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = c[i * RS];
            return v;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = r0 + i < R ? r0 + i : R - 1;
            const float x = col[r * RS];
            v[i] = r0 + i < R ? x : 0.f;
        }
        return v;
    } else {
        if (16 * m + 16 <= R) {
            f32x4 v;
            __builtin_memcpy(&v, col + r0, 16);
            return v;
        }
        const int rc = r0 + 4 <= R ? r0 : R - 4;     // first row loaded
        const int sh = r0 - rc;                       // own row i sits at i + sh
        f32x4 v;
        __builtin_memcpy(&v, col + rc, 16);
        f32x4 out;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float x = v[3];
            if (i + sh == 0) x = v[0];
            if (i + sh == 1) x = v[1];
            if (i + sh == 2) x = v[2];
            out[i] = (r0 + i < R) ? x : 0.f;
        }
        return out;
    }
}

template <int R, int RS = 1>
__device__ __forceinline__ void store_tile(float *col, int m, int G, f32x4 v)
{
    const int r0 = 16 * m + 4 * G;
    if constexpr (RS > 1) {
        float *c = col + r0 * RS;
        if (16 * m + 16 <= R) {
#pragma unroll
            for (int i = 0; i < 4; ++i) c[i * RS] = v[i];
            return;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (r0 + i < R) c[i * RS] = v[i];
    } else {
        if (r0 + 4 <= R) {
            __builtin_memcpy(col + r0, &v, 16);
            return;
        }
        if (r0 < R) col[r0] = v[0];
        if (r0 + 1 < R) col[r0 + 1] = v[1];
        if (r0 + 2 < R) col[r0 + 2] = v[2];
    }
}

// hi/lo split of the eight K values of one K step (tiles a and b).
struct Split {
    bf16x8 hi, lo;
};

__device__ __forceinline__ Split split8(f32x4 a, f32x4 b)
{
    Split s;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        s.hi[i] = (__bf16)a[i];
        s.hi[4 + i] = (__bf16)b[i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        s.lo[i] = (__bf16)(a[i] - (float)s.hi[i]);
        s.lo[4 + i] = (__bf16)(b[i] - (float)s.hi[4 + i]);
    }
    return s;
}

// A-operand fragment f of a generated table: hi and lo parts of this lane.
struct AFrag {
    bf16x8 hi, lo;
};

__device__ __forceinline__ AFrag load_frag(const unsigned int *data, int f, int lane)
{
    const u32x4 *p = reinterpret_cast<const u32x4 *>(data);
    AFrag a;
    a.hi = __builtin_bit_cast(bf16x8, p[(2 * f) * 64 + lane]);
    a.lo = __builtin_bit_cast(bf16x8, p[(2 * f + 1) * 64 + lane]);
    return a;
}

// C += A B with the three split products.
__device__ __forceinline__ f32x4 mfma3(const AFrag &a, const Split &b, f32x4 c)
{
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.hi, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.lo, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.lo, b.hi, c, 0, 0, 0);
    return c;
}

// Y[p][m] += sum_d Mat^d[tile m] (sum_slot star^d[p][q_slot] X[q_slot]) over
// the K steps s < KS of the input column X (TI tiles), for the output tiles
// m < TO.  Mat^d is family FAM (K-tilde or K-hat) of degree N; stl points to
// this lane's element star in LDS ([p][d][slot]).  Per (K step, direction)
// the fragments of all output tiles are loaded once and serve the 9 quantity
// columns, whose mixed input is formed and split one column at a time.
template <int N, int FAM, int TI, int TO, int KS>
__device__ __forceinline__ void star_mfma(const float *stl, const f32x4 (&X)[NQ][TI], f32x4 (&Y)[NQ][TO],
                                          int lane)
{
    using F = mft::Frag<N, FAM>;
    static_for<0, KS>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        static_for<0, 3>([&](auto dc) {
            constexpr int d = decltype(dc)::value;
            AFrag a[TO];
            static_for<0, TO>([&](auto mc) {
                constexpr int m = decltype(mc)::value;
                if constexpr (F::idx[d][m][s] >= 0) a[m] = load_frag(F::data(), F::idx[d][m][s], lane);
            });
            static_for<0, NQ>([&](auto pc) {
                constexpr int p = decltype(pc)::value;
                const float c0 = stl[p * 9 + d * 3 + 0], c1 = stl[p * 9 + d * 3 + 1],
                            c2 = stl[p * 9 + d * 3 + 2];
                f32x4 x0 = zero4(), x1 = zero4();
                if constexpr (2 * s < TI)
                    x0 = c0 * X[star_q(p, 0)][2 * s] + c1 * X[star_q(p, 1)][2 * s] + c2 * X[star_q(p, 2)][2 * s];
                if constexpr (2 * s + 1 < TI)
                    x1 = c0 * X[star_q(p, 0)][2 * s + 1] + c1 * X[star_q(p, 1)][2 * s + 1] +
                         c2 * X[star_q(p, 2)][2 * s + 1];
                const Split b = split8(x0, x1);
                static_for<0, TO>([&](auto mc) {
                    constexpr int m = decltype(mc)::value;
                    if constexpr (F::idx[d][m][s] >= 0) Y[p][m] = mfma3(a[m], b, Y[p][m]);
                });
            });
        });
    });
}

// Stage the packed star matrices of the wave's element slots in LDS
// ([slot][p][d][slot], 81 floats per element); slots past E repeat the last
// element.
template <bool FUSED>
__device__ __forceinline__ void stage_star(float *st, const float *star, const Tile<FUSED> &L)
{
    for (int i = L.lane; i < Tile<FUSED>::SLOTS * 81; i += 64) {
        const int64_t e = i / 81;
        const int64_t src = (L.base + (e < L.nvalid ? e : L.nvalid - 1)) * 81 + (i - e * 81);
        st[i] = star[src];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Predictor + time integral + face traces.
// T^0 = Q, T^{k+1} = dt/(k+1) sum_xi Kt^xi T^k star^xi^T, I = sum_k dt/(k+1) T^k;
// traces[e][s] = R^s^T I.  The scale factors dt/(k+1) are formed in FP64 and
// rounded once; I starts from dt*Q (FP64 product, rounded once) and the
// derivative terms (rows < C(N+2,3) only: the staircase) are added in FP32.
// ---------------------------------------------------------------------------
template <int N, int DL, int TI>
__device__ __forceinline__ void ck_rest(int lane, const float *stl, double dt, const f32x4 (&X)[NQ][TI],
                                        f32x4 (&Ih)[NQ][tiles(nb3(N - 1))])
{
    if constexpr (DL < N) {
        constexpr int BO = nb3(N - DL - 1), TO = tiles(BO), KS = ksteps(nb3(N - DL));
        f32x4 Y[NQ][TO];
#pragma unroll
        for (int p = 0; p < NQ; ++p)
#pragma unroll
            for (int m = 0; m < TO; ++m) Y[p][m] = zero4();
        star_mfma<N, mft::KT, TI, TO, KS>(stl, X, Y, lane);
        const float sc = (float)(dt / double(DL + 1)), si = (float)(dt / double(DL + 2));
#pragma unroll
        for (int p = 0; p < NQ; ++p)
#pragma unroll
            for (int m = 0; m < TO; ++m) {
                Y[p][m] *= sc;
                Ih[p][m] += si * Y[p][m];
            }
        ck_rest<N, DL + 1, TO>(lane, stl, dt, Y, Ih);
    }
}

// Predictor, time integral and face traces of one wave's tile (one wave per
// workgroup; element tiling: 16 elements per wave, fused tiling: one element
// and its 16 simulations per wave; the XCD-aware block order over tiles).
template <int N, bool FUSED>
__global__ void __launch_bounds__(64)
k_mstep_predict(int64_t E, double dt, const float *__restrict__ Q, const float *__restrict__ star,
                float *__restrict__ Iout, float *__restrict__ traces)
{
    using T = Tile<FUSED>;
    __shared__ float st[T::SLOTS * 81];
    const int64_t lb = dgk::logical_block();
    constexpr int RS = T::RS;
    constexpr int B = nb3(N), Bf = nb2(N), Bv = nb3(N - 1);
    constexpr int TB = tiles(B), TV = tiles(Bv), TF = tiles(Bf), KB = ksteps(B);
    const T L(E, lb);
    stage_star(st, star, L);
    const float *stl = st + L.slot * 81;
    // column q of this lane's element (and simulation) is qe + q * QS
    constexpr int QS = B * RS;
    const float *qe = L.template col<B>(Q, L.elem, 0);
    float *ie = L.template col<B>(Iout, L.elem, 0);
    f32x4 D0[NQ][TB];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int m = 0; m < TB; ++m) D0[q][m] = load_tile<B, RS>(qe + q * QS, m, L.G);
    // first derivative from Q
    f32x4 Y[NQ][TV];
#pragma unroll
    for (int p = 0; p < NQ; ++p)
#pragma unroll
        for (int m = 0; m < TV; ++m) Y[p][m] = zero4();
    star_mfma<N, mft::KT, TB, TV, KB>(stl, D0, Y, L.lane);
    // I = dt*Q: rows of tiles >= TV get no derivative term and are final
    f32x4 Ih[NQ][TV];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int m = 0; m < TB; ++m) {
            f32x4 v;
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = (float)(dt * (double)D0[q][m][r]);
            if (m < TV) Ih[q][m] = v;
            else if (L.active) store_tile<B, RS>(ie + q * QS, m, L.G, v);
        }
    {
        const float sc = (float)dt, si = (float)(dt / 2.0);
#pragma unroll
        for (int p = 0; p < NQ; ++p)
#pragma unroll
            for (int m = 0; m < TV; ++m) {
                Y[p][m] *= sc;
                Ih[p][m] += si * Y[p][m];
            }
    }
    ck_rest<N, 1, TV>(L.lane, stl, dt, Y, Ih);
    if (L.active) {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int m = 0; m < TV; ++m) store_tile<B, RS>(ie + q * QS, m, L.G, Ih[q][m]);
    }
    // face traces R^s^T I.  The tiles >= TV of I are dt*Q again, recomputed
    // from Q (read only, so no ordering against this wave's stores of I).
    // The pointer is laundered so that the compiler reloads them instead of
    // keeping the first loads of those tiles alive through the derivatives.
    const float *qr = qe;
    asm volatile("" : "+v"(qr));
    f32x4 It[NQ][TB];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int m = 0; m < TB; ++m) {
            if (m < TV) {
                It[q][m] = Ih[q][m];
            } else {
                const f32x4 x = load_tile<B, RS>(qr + q * QS, m, L.G);
#pragma unroll
                for (int r = 0; r < 4; ++r) It[q][m][r] = (float)(dt * (double)x[r]);
            }
        }
    using FR = mft::Frag<N, mft::RT>;
    static_for<0, 4>([&](auto sc) {
        constexpr int sf = decltype(sc)::value;
        AFrag a[TF][KB];
        static_for<0, TF>([&](auto mc) {
            static_for<0, KB>([&](auto kc) {
                constexpr int m = decltype(mc)::value, s = decltype(kc)::value;
                if constexpr (FR::idx[sf][m][s] >= 0) a[m][s] = load_frag(FR::data(), FR::idx[sf][m][s], L.lane);
            });
        });
        float *te = L.template tcol<Bf>(traces, L.elem, sf, 0);
        constexpr int TS = Bf * RS;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            f32x4 t[TF];
#pragma unroll
            for (int m = 0; m < TF; ++m) t[m] = zero4();
            static_for<0, KB>([&](auto kc) {
                constexpr int s = decltype(kc)::value;
                const Split b = split8(It[q][2 * s], 2 * s + 1 < TB ? It[q][2 * s + 1 < TB ? 2 * s + 1 : 0] : zero4());
                static_for<0, TF>([&](auto mc) {
                    constexpr int m = decltype(mc)::value;
                    if constexpr (FR::idx[sf][m][s] >= 0) t[m] = mfma3(a[m][s], b, t[m]);
                });
            });
            if (L.active) {
#pragma unroll
                for (int m = 0; m < TF; ++m)
                    store_tile<Bf, RS>(te + q * TS, m, L.G, t[m]);
            }
        }
    });
}

// ---------------------------------------------------------------------------
// Corrector: Q += sum_xi Kh^xi I star^xi^T
//              + sum_s Rh^s [ (R^s^T I) A+^s^T + f^h (R^j^T I^nu) A-^s^T ]
// with the face traces read from the predictor's output.  Per face, the
// neighbour's trace is re-parameterised by f^h on the matrix cores: with one
// element per column the three orientation matrices act on copies of the
// trace in which the columns of elements with another h are zero, into one
// accumulator; in the fused tiling h is the wave's and one matrix acts.  Then
// g = A+ x_own + A- x_nbr in FP64 per face row (rounded once) and one lift
// by Rh^s (both flux terms share it).
// ---------------------------------------------------------------------------
template <int N, bool FUSED>
__global__ void __launch_bounds__(64)
k_mstep_correct(int64_t E, const float *__restrict__ Iin, const float *__restrict__ traces,
                const float *__restrict__ star, const double *__restrict__ Ap, const double *__restrict__ Am,
                const int32_t *__restrict__ neigh, const uint8_t *__restrict__ face_rot, float *__restrict__ Q)
{
    using T = Tile<FUSED>;
    __shared__ float st[T::SLOTS * 81];
    __shared__ double sA[2 * T::SLOTS * 81];
    const int64_t lb = dgk::logical_block();
    constexpr int RS = T::RS, SLOTS = T::SLOTS;
    constexpr int B = nb3(N), Bf = nb2(N), Bv = nb3(N - 1);
    constexpr int TB = tiles(B), TV = tiles(Bv), TF = tiles(Bf), KV = ksteps(Bv);
    static_assert(Bf <= 32, "a face column must fit one K step");
    const T L(E, lb);
    stage_star(st, star, L);
    const float *stl = st + L.slot * 81;
    f32x4 acc[NQ][TB];
#pragma unroll
    for (int p = 0; p < NQ; ++p)
#pragma unroll
        for (int m = 0; m < TB; ++m) acc[p][m] = zero4();
    {
        // volume: only the rows of I below C(N+2,3) meet a non-zero column of Kh
        const float *ie = L.template col<B>(Iin, L.elem, 0);
        f32x4 X[NQ][TV];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int m = 0; m < TV; ++m) X[q][m] = load_tile<Bv, RS>(ie + q * B * RS, m, L.G);
        star_mfma<N, mft::KH, TV, TB, KV>(stl, X, acc, L.lane);
    }
    __builtin_amdgcn_sched_barrier(0);
    using FF = mft::Frag<N, mft::FH>;
    using FL = mft::Frag<N, mft::RH>;
    static_for<0, 4>([&](auto sc) {
        constexpr int sf = decltype(sc)::value;
        const int32_t nu_raw = neigh[L.elem * 4 + sf];
        const int64_t nu = (nu_raw >= 0 && nu_raw < E) ? nu_raw : -1;   // out of range: no neighbour
        const int fr = face_rot[L.elem * 4 + sf];
        const int j = fr & 3, h = fr >> 2;
        // this face's flux solvers of the wave's elements to LDS ([A+|A-][slot][81])
        __syncthreads();
        for (int i = L.lane; i < SLOTS * 81; i += 64) {
            const int e = i / 81, k = i - e * 81;
            const int64_t el = L.base + (e < L.nvalid ? e : L.nvalid - 1);
            sA[i] = Ap[(el * 4 + sf) * 81 + k];
            sA[SLOTS * 81 + i] = Am[(el * 4 + sf) * 81 + k];
        }
        __syncthreads();
        const float *to = L.template tcol<Bf>(traces, L.elem, sf, 0);
        const float *tn = L.template tcol<Bf>(traces, nu >= 0 ? nu : 0, j, 0);
        f32x4 xo[NQ][TF], xn[NQ][TF];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int m = 0; m < TF; ++m) {
                xo[q][m] = load_tile<Bf, RS>(to + q * Bf * RS, m, L.G);
                xn[q][m] = nu >= 0 ? load_tile<Bf, RS>(tn + q * Bf * RS, m, L.G) : zero4();
            }
        // orientation: xn <- f^h xn (one K step: Bf <= 32), column by column
        // (the oriented column replaces the read one)
        if constexpr (FUSED) {
            AFrag fa[TF];
            static_for<0, TF>([&](auto mc) {
                constexpr int m = decltype(mc)::value;
                const int f = h == 0 ? FF::idx[0][m][0] : (h == 1 ? FF::idx[1][m][0] : FF::idx[2][m][0]);
                if (f >= 0) fa[m] = load_frag(FF::data(), f, L.lane);
            });
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                f32x4 o[TF];
#pragma unroll
                for (int m = 0; m < TF; ++m) o[m] = zero4();
                const Split b = split8(xn[q][0], TF > 1 ? xn[q][TF > 1 ? 1 : 0] : zero4());
#pragma unroll
                for (int m = 0; m < TF; ++m) o[m] = mfma3(fa[m], b, o[m]);
#pragma unroll
                for (int m = 0; m < TF; ++m) xn[q][m] = o[m];
            }
        } else {
            AFrag fa[3][TF];
            static_for<0, 3>([&](auto hc) {
                static_for<0, TF>([&](auto mc) {
                    constexpr int hh = decltype(hc)::value, m = decltype(mc)::value;
                    if constexpr (FF::idx[hh][m][0] >= 0) fa[hh][m] = load_frag(FF::data(), FF::idx[hh][m][0], L.lane);
                });
            });
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                f32x4 o[TF];
#pragma unroll
                for (int m = 0; m < TF; ++m) o[m] = zero4();
                const f32x4 a0 = xn[q][0], a1 = TF > 1 ? xn[q][TF > 1 ? 1 : 0] : zero4();
                static_for<0, 3>([&](auto hc) {
                    constexpr int hh = decltype(hc)::value;
                    const bool mine = h == hh;
                    const Split b = split8(mine ? a0 : zero4(), mine ? a1 : zero4());
                    static_for<0, TF>([&](auto mc) {
                        constexpr int m = decltype(mc)::value;
                        if constexpr (FF::idx[hh][m][0] >= 0) o[m] = mfma3(fa[hh][m], b, o[m]);
                    });
                });
#pragma unroll
                for (int m = 0; m < TF; ++m) xn[q][m] = o[m];
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        // per quantity p: g = A+ xo + A- xn per face row in FP64 (rounded
        // once), split, and lifted by Rh^s into every output tile
        AFrag la[TB];
        static_for<0, TB>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            if constexpr (FL::idx[sf][m][0] >= 0) la[m] = load_frag(FL::data(), FL::idx[sf][m][0], L.lane);
        });
        const double *ap = sA + L.slot * 81, *am = sA + (SLOTS + L.slot) * 81;
        // three quantities p at a time: the FP64 copies of one trace column
        // serve three rows of A+/A-; kept across all nine they would take
        // twice the traces' registers
        static_for<0, 3>([&](auto pgc) {
            constexpr int p0 = 3 * decltype(pgc)::value;
#pragma unroll
            for (int q = 0; q < NQ; ++q)
#pragma unroll
                for (int m = 0; m < TF; ++m) asm volatile("" : "+v"(xo[q][m]), "+v"(xn[q][m]));
            double gp[3][TF][4];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int m = 0; m < TF; ++m)
#pragma unroll
                    for (int r = 0; r < 4; ++r) gp[i][m][r] = 0.0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                __builtin_amdgcn_sched_barrier(0);
                double xd[TF][4], nd[TF][4];
#pragma unroll
                for (int m = 0; m < TF; ++m)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        xd[m][r] = (double)xo[q][m][r];
                        nd[m][r] = (double)xn[q][m][r];
                    }
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const double a = ap[(p0 + i) * 9 + q], b = am[(p0 + i) * 9 + q];
#pragma unroll
                    for (int m = 0; m < TF; ++m)
#pragma unroll
                        for (int r = 0; r < 4; ++r) gp[i][m][r] = fma(a, xd[m][r], fma(b, nd[m][r], gp[i][m][r]));
                }
            }
            static_for<0, 3>([&](auto ic) {
                constexpr int i = decltype(ic)::value, p = p0 + i;
                f32x4 g0, g1 = zero4();
#pragma unroll
                for (int r = 0; r < 4; ++r) g0[r] = (float)gp[i][0][r];
                if constexpr (TF > 1) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) g1[r] = (float)gp[i][TF > 1 ? 1 : 0][r];
                }
                const Split g = split8(g0, g1);
                static_for<0, TB>([&](auto mc) {
                    constexpr int m = decltype(mc)::value;
                    if constexpr (FL::idx[sf][m][0] >= 0) acc[p][m] = mfma3(la[m], g, acc[p][m]);
                });
            });
            __builtin_amdgcn_sched_barrier(0);
        });
        __builtin_amdgcn_sched_barrier(0);
    });
    if (L.active) {
        float *qe = L.template col<B>(Q, L.elem, 0);
#pragma unroll
        for (int p = 0; p < NQ; ++p)
#pragma unroll
            for (int m = 0; m < TB; ++m) {
                const f32x4 v = load_tile<B, RS>(qe + p * B * RS, m, L.G) + acc[p][m];
                store_tile<B, RS>(qe + p * B * RS, m, L.G, v);
            }
    }
}

}  // namespace dgm
