// Element-local ADER-DG kernels for the elastic wave equation on tetrahedra
// (paper Sec. 5.1.1, Eqs. seissol:derivative, seissol:timeint,
// seissol:correction_local, seissol:correction_neigh), written for CDNA4.
//
// Work decomposition: one 64-lane wavefront per workgroup handles 7
// elements; lane = (element e, quantity p), lane 63 shadows element 7 and
// never stores.  A lane owns one column (basis coefficients of quantity p)
// of its element.  Contractions with the element-independent reference
// matrices act column-wise and run as fully unrolled FP64/FP32 FMAs whose
// matrix operand is a compile-time literal (generated from the sparsity of
// each matrix, so structural zeros cost nothing and the matrices need no
// memory traffic).  Contractions over the
// quantity index (star matrices, flux solvers) mix columns; those go through
// an LDS chunk buffer (32 or 64 rows per column).  All global traffic of element-major arrays is
// staged through the same buffer so that it is fully coalesced.
//
// Arrays are element major: Q, I [E][9][B]; T [E][N+1][9][B] (Taylor-scaled
// derivatives dt^d/d! D^d); traces [E][4][9][Bf]; packed star [E][9][3][3];
// flux solvers A+/A- [E][4][9][9] FP64.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#include "dg_common.h"
#include "dg_generated.h"

namespace dgk {

constexpr int EPW = 7;     // elements per wavefront
constexpr int NQ = 9;      // elastic quantities
#ifndef DG_DEGREE
#error "DG_DEGREE (the polynomial degree of this translation unit) must be defined"
#endif
// Rows per LDS chunk (LDS budget: 19 KB per one-wave workgroup in FP64,
// 9.5 KB in FP32); 32 rows hold every face-basis column (Bf <= 28).
template <typename real>
constexpr int CH = 32;
template <typename real>
constexpr int LB = CH<real> + 1;   // padded (odd) row stride of a column in LDS
constexpr int NCOL = 8 * NQ;


// q-columns read by row p of the packed star matrix (elastic pattern:
// stress rows couple to velocities, velocity rows to stresses)
__device__ __forceinline__ void star_cols(int p, int &q0, int &q1, int &q2)
{
    switch (p) {
    case 0: case 1: case 2: q0 = 6; q1 = 7; q2 = 8; break;
    case 3: q0 = 6; q1 = 7; q2 = 6; break;
    case 4: q0 = 7; q1 = 8; q2 = 7; break;
    case 5: q0 = 6; q1 = 8; q2 = 6; break;
    case 6: q0 = 0; q1 = 3; q2 = 5; break;
    case 7: q0 = 1; q1 = 3; q2 = 4; break;
    default: q0 = 2; q1 = 4; q2 = 5; break;
    }
}

template <typename real>
struct Lane {
    int lane, e, p;
    int64_t base, elem;
    bool active;
    real *buf;      // LDS chunk buffer [8][9][LB<real>]
    real *own;      // this lane's column in buf
};


template <typename real>
__device__ __forceinline__ Lane<real> make_lane(real *buf, int64_t E, int64_t lb)
{
    Lane<real> L;
    L.lane = threadIdx.x;
    L.e = L.lane / NQ;
    L.p = L.lane - L.e * NQ;
    L.base = lb * EPW;
    const int64_t el = L.base + L.e;
    L.active = (L.e < EPW) && (el < E);
    L.elem = el < E ? el : E - 1;
    L.buf = buf;
    L.own = buf + (L.e * NQ + L.p) * LB<real>;
    return L;
}

__device__ __forceinline__ void lds_sync() { __syncthreads(); }

// Scheduling fence every SB rows of an unrolled contraction: keeps the
// scheduler from hoisting a whole chunk's LDS reads above its FMAs, which
// would cost one register pair per hoisted value.
constexpr int SB = 4;
template <int R>
__device__ __forceinline__ void row_fence()
{
    if constexpr (R % SB == SB - 1) __builtin_amdgcn_sched_barrier(0);
}

// Condition of a code block that always runs.  In FP64 the value is opaque
// to the compiler, so every block is a basic block of its own and the
// compiler materialises the literal matrix entries per block instead of
// keeping each distinct value in a scalar register across the whole kernel
// (which overflows the scalar file into vector-lane spills).
template <typename real>
__device__ __forceinline__ bool code_block()
{
    if constexpr (sizeof(real) == 8) {
        int v;
        asm volatile("s_mov_b32 %0, 1" : "=s"(v));
        return v != 0;
    } else {
        return true;
    }
}

// element of slot g (0..7) of this wave, clamped into range
__device__ __forceinline__ int64_t slot_elem(int64_t base, int g, int64_t E)
{
    const int64_t el = base + g;
    return el < E ? el : E - 1;
}

// Rows of a missing element (no neighbour) are read from here: zero-filled
// static storage, longer than any element block.
__device__ double dg_zero_block[1024];

// Lanes move element data in groups of 8: lane (g, s) = (lane / 8, lane % 8)
// handles rows s, s+8, ... of the 9 columns of element slot g, so every
// global and LDS address is the lane's base plus a compile-time offset (no
// per-value index arithmetic); the 8 lanes of a group touch 8 consecutive
// values of one column.
template <int CNT>
struct RowSplit {
    static constexpr int K = (CNT + 7) / 8;          // rows per lane and column
    static constexpr int TAIL = CNT - 8 * (K - 1);   // lanes s < TAIL own row 8(K-1)+s
};

// One chunk of element data in flight: rows [l0, l0+CNT) of the 9 columns of
// this lane's element slot, K values per column.
template <int CNT, typename real>
struct ChunkRegs {
    real v[NQ][RowSplit<CNT>::K];
};

// Issue the loads of a chunk (rows [l0, l0+CNT) of the 9 columns of every
// element slot).  eptr(g) is the global address of row 0 of column 0 of slot
// g's element block, whose columns are QS apart, or null for zeros.  All
// loads of the chunk are in flight together.  Branch free: in the last row
// of a column, lanes past the chunk re-read its row 0 (chunk_put then writes
// them to rows [CNT, 8K) of their LDS column, which nothing reads).
template <int CNT, int QS, typename real, typename EPtr>
__device__ __forceinline__ ChunkRegs<CNT, real> chunk_fetch(const Lane<real> &L, EPtr eptr, int l0)
{
    using RS = RowSplit<CNT>;
    constexpr int K = RS::K;
    static_assert(8 * K <= LB<real>, "tail rows must stay inside the column slot");
    static_assert(9 * QS <= 1024, "element block longer than the zero block");
    const int g = L.lane >> 3, s = L.lane & 7;
    const real *e0 = eptr(g);
    const real *src = (e0 ? e0 : reinterpret_cast<const real *>(dg_zero_block)) + l0 + s;
    const real *srct = s < RS::TAIL ? src + 8 * (K - 1) : src - s;   // last row, else row 0
    ChunkRegs<CNT, real> r;
    static_for<0, NQ>([&](auto qi) {
        static_for<0, K>([&](auto ki) {
            constexpr int q = decltype(qi)::value, kk = decltype(ki)::value;
            r.v[q][kk] = kk < K - 1 ? src[q * QS + 8 * kk] : srct[q * QS];
        });
    });
    return r;
}

// Two fetched chunks (own and neighbour face rows of the corrector).
template <int CNT, typename real>
struct ChunkPair {
    ChunkRegs<CNT, real> xo, xn;
};

// Write a fetched chunk to LDS (slot g, column q, row r at
// buf[(g*NQ + q)*LB + r]).
template <int CNT, typename real>
__device__ __forceinline__ void chunk_put(const Lane<real> &L, const ChunkRegs<CNT, real> &r)
{
    constexpr int K = RowSplit<CNT>::K;
    const int g = L.lane >> 3, s = L.lane & 7;
    real *dst = L.buf + g * NQ * LB<real> + s;
    static_for<0, NQ>([&](auto qi) {
        static_for<0, K>([&](auto ki) {
            constexpr int q = decltype(qi)::value, kk = decltype(ki)::value;
            dst[q * LB<real> + 8 * kk] = r.v[q][kk];
        });
    });
    __builtin_amdgcn_sched_barrier(0);
}

// Cooperative load of a chunk into LDS: one memory round trip.
template <int CNT, int QS, typename real, typename EPtr>
__device__ __forceinline__ void chunk_load(const Lane<real> &L, EPtr eptr, int l0)
{
    chunk_put<CNT>(L, chunk_fetch<CNT, QS>(L, eptr, l0));
}

// Cooperative store of rows [l0, l0+CNT) of the columns of the real
// (non-shadow, in-range) element slots from LDS; eptr as for chunk_load.
template <int CNT, int QS, typename real, typename EPtr>
__device__ __forceinline__ void chunk_store(const Lane<real> &L, EPtr eptr, int l0, int64_t E)
{
    using RS = RowSplit<CNT>;
    constexpr int K = RS::K;
    const int g = L.lane >> 3, s = L.lane & 7;
    if (g < EPW && L.base + g < E) {
        real *dst = eptr(g) + l0 + s;
        const real *src = L.buf + g * NQ * LB<real> + s;
        static_for<0, NQ>([&](auto qi) {
            static_for<0, K - 1>([&](auto ki) {
                constexpr int q = decltype(qi)::value, kk = decltype(ki)::value;
                dst[q * QS + 8 * kk] = src[q * LB<real> + 8 * kk];
            });
            __builtin_amdgcn_sched_barrier(0);
        });
        if (s < RS::TAIL) {
            static_for<0, NQ>([&](auto qi) {
                constexpr int q = decltype(qi)::value;
                dst[q * QS + 8 * (K - 1)] = src[q * LB<real> + 8 * (K - 1)];
            });
        }
    }
}

// load this lane's own column (rows [0,R)) of an element-major array into regs
template <int R, int QS, typename real, typename EPtr>
__device__ __forceinline__ void load_columns(const Lane<real> &L, EPtr eptr, real *dst)
{
    static_for<0, (R + CH<real> - 1) / CH<real>>([&](auto ci) {
        constexpr int l0 = decltype(ci)::value * CH<real>;
        constexpr int cnt = (R - l0) < CH<real> ? (R - l0) : CH<real>;
        chunk_load<cnt, QS>(L, eptr, l0);
        lds_sync();
        static_for<0, cnt>([&](auto ri) { dst[l0 + ri] = L.own[ri]; });
        lds_sync();
    });
}

// Cooperative store of zeros to rows [l0, l0+CNT) of the columns of the real
// element slots, in chunk_store's pattern but with no LDS source.
template <int CNT, int QS, typename real, typename EPtr>
__device__ __forceinline__ void chunk_zero(const Lane<real> &L, EPtr eptr, int l0, int64_t E)
{
    using RS = RowSplit<CNT>;
    constexpr int K = RS::K;
    const int g = L.lane >> 3, s = L.lane & 7;
    if (g < EPW && L.base + g < E) {
        real *dst = eptr(g) + l0 + s;
        static_for<0, NQ>([&](auto qi) {
            static_for<0, K - 1>([&](auto ki) {
                constexpr int q = decltype(qi)::value, kk = decltype(ki)::value;
                dst[q * QS + 8 * kk] = real(0);
            });
        });
        if (s < RS::TAIL) {
            static_for<0, NQ>([&](auto qi) {
                constexpr int q = decltype(qi)::value;
                dst[q * QS + 8 * (K - 1)] = real(0);
            });
        }
    }
}

// store this lane's own column rows [0,R) from regs (rows >= RV written as
// 0; chunks that hold only such rows are written directly, without LDS)
template <int R, int RV, int QS, typename real, typename EPtr>
__device__ __forceinline__ void store_columns(const Lane<real> &L, EPtr eptr, const real *src, int64_t E)
{
    static_for<0, (R + CH<real> - 1) / CH<real>>([&](auto ci) {
        constexpr int l0 = decltype(ci)::value * CH<real>;
        constexpr int cnt = (R - l0) < CH<real> ? (R - l0) : CH<real>;
        if constexpr (l0 >= RV) {
            chunk_zero<cnt, QS>(L, eptr, l0, E);
        } else {
            static_for<0, cnt>([&](auto ri) {
                constexpr int l = l0 + decltype(ri)::value;
                if constexpr (l < RV) L.own[ri] = src[l];
                else L.own[ri] = real(0);
            });
            lds_sync();
            chunk_store<cnt, QS>(L, eptr, l0, E);
            lds_sync();
        }
    });
}

// store rows [M0, M0+CNT) of this lane's register column to rows [0, CNT) of
// element blocks whose columns are CNT apart (one part of a face block)
template <int M0, int CNT, typename real, typename EPtr>
__device__ __forceinline__ void store_part(const Lane<real> &L, EPtr eptr, const real *src, int64_t E)
{
    static_for<0, CNT>([&](auto ri) { L.own[ri] = src[M0 + decltype(ri)::value]; });
    lds_sync();
    chunk_store<CNT, CNT>(L, eptr, 0, E);
    lds_sync();
}

// Q(own column) += acc, rows [0,B)
template <int B, typename real>
__device__ __forceinline__ void add_to_q(const Lane<real> &L, real *Q, const real *acc, int64_t E)
{
    auto blk = [&](int g) { return Q + slot_elem(L.base, g, E) * NQ * B; };
    auto cblk = [&](int g) -> const real * { return blk(g); };
    constexpr int NCH = (B + CH<real> - 1) / CH<real>;
    auto update = [&](auto l0c) {
        constexpr int l0 = decltype(l0c)::value, cnt = (B - l0) < CH<real> ? (B - l0) : CH<real>;
        lds_sync();
        static_for<0, cnt>([&](auto ri) { L.own[ri] += acc[l0 + ri]; });
        lds_sync();
        chunk_store<cnt, B>(L, blk, l0, E);
        lds_sync();
    };
    if constexpr (NCH == 2) {
        // two chunks: both chunks' loads in flight together (one memory round
        // trip, and no line shared by the two chunks is fetched twice; their
        // registers fit beside the accumulators)
        constexpr int c1 = B - CH<real>;
        const auto r0 = chunk_fetch<CH<real>, B>(L, cblk, 0);
        const auto r1 = chunk_fetch<c1, B>(L, cblk, CH<real>);
        chunk_put<CH<real>>(L, r0);
        update(std::integral_constant<int, 0>{});
        chunk_put<c1>(L, r1);
        update(std::integral_constant<int, CH<real>>{});
    } else {
        static_for<0, NCH>([&](auto ci) {
            constexpr int l0 = decltype(ci)::value * CH<real>;
            constexpr int cnt = (B - l0) < CH<real> ? (B - l0) : CH<real>;
            chunk_load<cnt, B>(L, cblk, l0);
            update(std::integral_constant<int, l0>{});
        });
    }
}

template <typename real>
struct Star {
    real s[3][3];   // [d][slot]
    int q0, q1, q2;
};

template <typename real>
__device__ __forceinline__ Star<real> load_star(const Lane<real> &L, const real *star_packed)
{
    Star<real> S;
    star_cols(L.p, S.q0, S.q1, S.q2);
    const real *sp = star_packed + (L.elem * NQ + L.p) * 9;
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int i = 0; i < 3; ++i) S.s[d][i] = sp[d * 3 + i];
    return S;
}

// acc[k] += sum_d K^d[k][l] (sum_q star^d[p][q] X[l][q]) for rows l in
// [0, NROWS) whose values sit in LDS chunk-wise; `fill(l0, cnt)` brings rows
// [l0, l0+cnt) of all column slots into LDS.
template <int N, bool KTILDE, int NROWS, bool BLOCKS = true, typename real, typename Fill>
__device__ __forceinline__ void star_contract(const Lane<real> &L, const Star<real> &S, real *acc, Fill fill)
{
    static_for<0, (NROWS + CH<real> - 1) / CH<real>>([&](auto ci) {
        constexpr int l0 = decltype(ci)::value * CH<real>;
        constexpr int cnt = (NROWS - l0) < CH<real> ? (NROWS - l0) : CH<real>;
        fill(std::integral_constant<int, l0>{}, std::integral_constant<int, cnt>{});
        lds_sync();
        const real *b0 = L.buf + (L.e * NQ + S.q0) * LB<real>;
        const real *b1 = L.buf + (L.e * NQ + S.q1) * LB<real>;
        const real *b2 = L.buf + (L.e * NQ + S.q2) * LB<real>;
        static_for<0, (cnt + SB - 1) / SB>([&](auto bi) {
            constexpr int r0 = decltype(bi)::value * SB, rn = (cnt - r0) < SB ? (cnt - r0) : SB;
            if (!BLOCKS || code_block<real>()) {
                static_for<0, rn>([&](auto rj) {
                    constexpr int ri = r0 + decltype(rj)::value, l = l0 + ri;
                    const real v0 = b0[ri], v1 = b1[ri], v2 = b2[ri];
                    const real x0 = fma(S.s[0][0], v0, fma(S.s[0][1], v1, S.s[0][2] * v2));
                    const real x1 = fma(S.s[1][0], v0, fma(S.s[1][1], v1, S.s[1][2] * v2));
                    const real x2 = fma(S.s[2][0], v0, fma(S.s[2][1], v1, S.s[2][2] * v2));
                    if constexpr (KTILDE) KtCol<N, l>::apply(x0, x1, x2, acc);
                    else KhCol<N, l>::apply(x0, x1, x2, acc);
                });
            }
            __builtin_amdgcn_sched_barrier(0);
        });
        lds_sync();
    });
}

// acc[k] += sum_m Rh^S[k][m] sum_q A[p][q] X[m][q] for face rows m in [0,Bf)
// with X chunk-wise in LDS (fill brings rows in).
template <int N, int S, bool MIX = false, typename real, typename Fill>
__device__ __forceinline__ void flux_lift(const Lane<real> &L, const double *A, real *acc, Fill fill)
{
    // MIX: the flux-solver product runs in FP64 (FP64 matrices, FP32 traces),
    // rounded once before the FP32 lift
    using mreal = typename std::conditional<MIX, double, real>::type;
    constexpr int Bf = nb2(N);
    mreal a[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) a[q] = (mreal)A[L.p * NQ + q];
    const real *xe = L.buf + L.e * NQ * LB<real>;
    static_for<0, (Bf + CH<real> - 1) / CH<real>>([&](auto ci) {
        constexpr int m0 = decltype(ci)::value * CH<real>;
        constexpr int cnt = (Bf - m0) < CH<real> ? (Bf - m0) : CH<real>;
        fill(std::integral_constant<int, m0>{}, std::integral_constant<int, cnt>{});
        lds_sync();
        static_for<0, cnt>([&](auto ri) {
            constexpr int m = m0 + decltype(ri)::value;
            mreal g = a[0] * (mreal)xe[ri];
#pragma unroll
            for (int q = 1; q < NQ; ++q) g = fma(a[q], (mreal)xe[q * LB<real> + ri], g);
            RhCol<N, S, m>::apply((real)g, acc);
            row_fence<decltype(ri)::value>();
        });
        lds_sync();
    });
}

// Face rows in parts of whole degree blocks (degree d holds rows
// [d(d+1)/2, (d+1)(d+2)/2)), each part at most fpr rows.  With fpr = 16 the
// own and the neighbour rows of one part fit side by side in one LDS chunk
// (used in FP64, where a second chunk buffer would halve occupancy).
template <typename real>
constexpr int FPR = sizeof(real) == 8 ? 16 : 64;
__host__ __device__ constexpr int face_parts(int n, int fpr)
{
    int parts = 1, rows = 0;
    for (int d = 0; d <= n; ++d) {
        if (rows + d + 1 > fpr) { ++parts; rows = 0; }
        rows += d + 1;
    }
    return parts;
}
// first degree of part i (the last part ends at degree n + 1)
__host__ __device__ constexpr int face_part_d0(int n, int fpr, int i)
{
    int part = 0, rows = 0;
    for (int d = 0; d <= n; ++d) {
        if (rows + d + 1 > fpr) { ++part; rows = 0; }
        if (part == i && rows == 0) return d;
        rows += d + 1;
    }
    return n + 1;
}

// col[m - M0] <- sum_n f^h[m][n] col[n - M0] for the degree blocks
// [D0, D1) of one face-basis column in LDS (rows from M0 = D0(D0+1)/2 on);
// f^h is block diagonal by degree and is applied one block at a time.
template <int N, int D0, int D1, typename real>
__device__ __forceinline__ void orient_column(real *col, int h)
{
    constexpr int M0 = D0 * (D0 + 1) / 2;
    static_for<D0, D1>([&](auto di) {
        constexpr int d = decltype(di)::value, off = d * (d + 1) / 2 - M0;
        real in[d + 1], out[d + 1];
#pragma unroll
        for (int i = 0; i < d + 1; ++i) in[i] = col[off + i];
        if (h == 0) FBlock<N, 0, d>::apply(in, out);
        else if (h == 1) FBlock<N, 1, d>::apply(in, out);
        else FBlock<N, 2, d>::apply(in, out);
#pragma unroll
        for (int i = 0; i < d + 1; ++i) col[off + i] = out[i];
    });
}

// Both flux terms of face S, rows [M0, M0+CNT) of the face basis, with one
// lift:
// acc[k] += sum_m Rh^S[k][m] sum_q (Ap[p][q] Xo[m][q] + Am[p][q] Xn[m][q]),
// with those rows of the own traces Xo and of the (already oriented)
// neighbour traces Xn in LDS (columns of xo_buf and xn_buf, row m at m - M0,
// row stride LB).  The local and neighbour terms are lifted by the same
// matrix, so summing before the lift halves the lift work.  MIX: the sum
// runs in FP64 and is rounded once before the FP32 lift.
template <int N, int S, bool MIX, int M0, int CNT, typename real>
__device__ __forceinline__ void flux_lift_pair(const Lane<real> &L, const double *Ap, const double *Am,
                                               const real *xo_buf, const real *xn_buf, real *acc)
{
    using mreal = typename std::conditional<MIX, double, real>::type;
    mreal ap[NQ], am[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        ap[q] = (mreal)Ap[L.p * NQ + q];
        am[q] = (mreal)Am[L.p * NQ + q];
    }
    const real *xo = xo_buf + L.e * NQ * LB<real>;
    const real *xn = xn_buf + L.e * NQ * LB<real>;
    // rows per code block: each row reads 18 LDS values, which the scheduler
    // issues ahead for the whole block; in FP64 two rows keep that in budget
    constexpr int SBL = sizeof(real) == 8 ? 2 : SB;
    static_for<0, (CNT + SBL - 1) / SBL>([&](auto bi) {
        constexpr int r0 = decltype(bi)::value * SBL, rn = (CNT - r0) < SBL ? (CNT - r0) : SBL;
        if (code_block<real>()) {
            static_for<0, rn>([&](auto rj) {
                constexpr int r = r0 + decltype(rj)::value;
                mreal g = ap[0] * (mreal)xo[r];
#pragma unroll
                for (int q = 1; q < NQ; ++q) g = fma(ap[q], (mreal)xo[q * LB<real> + r], g);
#pragma unroll
                for (int q = 0; q < NQ; ++q) g = fma(am[q], (mreal)xn[q * LB<real> + r], g);
                RhCol<N, S, M0 + r>::apply((real)g, acc);
            });
        }
        __builtin_amdgcn_sched_barrier(0);
    });
}

template <int N, int S, typename real>
__device__ __forceinline__ void face_trace(const real *I, real *tr)
{
    constexpr int B = nb3(N), Bf = nb2(N);
#pragma unroll
    for (int m = 0; m < Bf; ++m) tr[m] = real(0);
    static_for<0, (B + 7) / 8>([&](auto bi) {
        constexpr int l0 = decltype(bi)::value * 8, ln = (B - l0) < 8 ? (B - l0) : 8;
        if (code_block<real>()) {
            static_for<0, ln>([&](auto lj) {
                constexpr int l = l0 + decltype(lj)::value;
                RCol<N, S, l>::apply(I[l], tr);
            });
        }
        __builtin_amdgcn_sched_barrier(0);
    });
}

template <int N, typename real>
__device__ __forceinline__ void orient_rt(int h, const real *in, real *out)
{
    if (h == 0) FApply<N, 0>::apply(in, out);
    else if (h == 1) FApply<N, 1>::apply(in, out);
    else FApply<N, 2>::apply(in, out);
}

// ---------------------------------------------------------------------------
// Predictor (Eq. seissol:derivative) with the time integral (Eq.
// seissol:timeint) accumulated on the fly.  T^0 = Q,
// T^{d+1} = dt/(d+1) sum_xi Kt^xi T^d star^xi^T,  I = sum_d dt/(d+1) T^d.
// ---------------------------------------------------------------------------
// ireal: type of the time-integral accumulator (FP64 in the mixed form).
// ALIAS: src and I are the same array (T^0 = Q accumulates into I in place).
template <int N, int D, bool WRITE_T, bool ACC_I, bool ALIAS, typename real, typename ireal, typename TColPtr>
__device__ __forceinline__ void ck_recurse(const Lane<real> &L, const Star<real> &S, ireal dt, real *src,
                                           ireal *I, TColPtr tblk, int64_t E)
{
    constexpr int B = nb3(N);
    if constexpr (D < N) {
        constexpr int bin = nb3(N - D), bout = nb3(N - D - 1);
        real acc[bout];
#pragma unroll
        for (int k = 0; k < bout; ++k) acc[k] = real(0);
        star_contract<N, true, bin>(L, S, acc, [&](auto l0c, auto cntc) {
            constexpr int l0 = decltype(l0c)::value, cnt = decltype(cntc)::value;
            static_for<0, cnt>([&](auto ri) { L.own[ri] = src[l0 + ri]; });
        });
        if constexpr (ACC_I && D == 0) {
#pragma unroll
            for (int k = 0; k < B; ++k) {
                if constexpr (ALIAS) I[k] *= dt;          // src aliases I: T^0 = Q
                else I[k] = dt * (ireal)src[k];
            }
        }
        const real sc = real(dt / ireal(D + 1));
        const ireal si = dt / ireal(D + 2);
#pragma unroll
        for (int k = 0; k < bout; ++k) {
            acc[k] *= sc;
            if constexpr (ACC_I) I[k] = fma(si, (ireal)acc[k], I[k]);
        }
        if constexpr (WRITE_T) store_columns<B, bout, B>(L, [&](int g) { return tblk(g, D + 1); }, acc, E);
        ck_recurse<N, D + 1, WRITE_T, ACC_I, ALIAS>(L, S, dt, acc, I, tblk, E);
    }
}

// Per-stage predictor (Eq. seissol:derivative) in one launch: T^0 = Q is
// copied while Q streams in, then each order
// T^{D+1} = dt/(D+1) sum_xi Kt^xi T^D star^xi^T is formed from the previous
// one held in registers and written as it is formed (rows past the staircase
// as 0).  Each order reads the same values in the same order as a launch per
// order reading T^D back from memory would, so T is the same to the bit.
template <int N, typename real>
__global__ void __launch_bounds__(64) k_predictor(int64_t E, real dt, const real *__restrict__ Q,
                                                  const real *__restrict__ star, real *__restrict__ T)
{
    constexpr int B = nb3(N);
    __shared__ real buf[NCOL * LB<real>];
    const Lane<real> L = make_lane(buf, E, logical_block());
    const Star<real> S = load_star(L, star);
    auto tblk = [&](int g, int d) { return T + (slot_elem(L.base, g, E) * (N + 1) + d) * NQ * B; };
    auto qblk = [&](int g) -> const real * { return Q + slot_elem(L.base, g, E) * NQ * B; };
    real q[B];
    static_for<0, (B + CH<real> - 1) / CH<real>>([&](auto ci) {
        constexpr int l0 = decltype(ci)::value * CH<real>;
        constexpr int cnt = (B - l0) < CH<real> ? (B - l0) : CH<real>;
        chunk_load<cnt, B>(L, qblk, l0);
        lds_sync();
        chunk_store<cnt, B>(L, [&](int g) { return tblk(g, 0); }, l0, E);
        static_for<0, cnt>([&](auto ri) { q[l0 + ri] = L.own[ri]; });
        lds_sync();
    });
    ck_recurse<N, 0, true, false, false>(L, S, dt, q, static_cast<real *>(nullptr), tblk, E);
}

// Time integral over stored Taylor-scaled derivatives (FP64 accumulation).
// Each derivative lowers the polynomial degree by one, so T^d vanishes in the
// hierarchical basis rows at and past nb3(N - d); those rows add nothing to
// the sum and are not read.  Skipped rows are contiguous runs at the end of
// each quantity column, so the lines they occupy are never fetched: at degree
// 5 the bytes per element drop from 7 column blocks to about 3.3.
template <int N, typename real>
__global__ void __launch_bounds__(256) k_time_integral(int64_t E, double dt, const real *__restrict__ T,
                                                       real *__restrict__ I)
{
    constexpr int B = nb3(N);
    const int64_t n = E * NQ * B;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = i / (NQ * B), r = i - e * (NQ * B);
        const int k = (int)(r - (r / B) * B);   // basis row
        const real *t = T + e * (N + 1) * NQ * B + r;
        double s = 0.0;
#pragma unroll
        for (int d = 0; d <= N; ++d)
            if (k < nb3(N - d)) s = fma(dt / double(d + 1), (double)t[d * NQ * B], s);
        I[i] = (real)s;
    }
}

// Volume term: Q += sum_xi Kh^xi I star^xi^T
template <int N, typename real>
__device__ __forceinline__ void volume_acc(const Lane<real> &L, const Star<real> &S, const real *I, real *acc, int64_t E)
{
    constexpr int B = nb3(N), Bv = nb3(N - 1);
    auto iblk = [&](int g) -> const real * { return I + slot_elem(L.base, g, E) * NQ * B; };
    if constexpr ((sizeof(real) == 4 || N <= 5) && (Bv + CH<real> - 1) / CH<real> == 2) {
        // two chunks: the second chunk's loads are issued with the first, so
        // their latency overlaps the first chunk's contraction (not for FP64
        // at degree 6, whose registers are already exhausted)
        constexpr int c1 = Bv - CH<real>;
        const auto r0 = chunk_fetch<CH<real>, B>(L, iblk, 0);
        const auto r1 = chunk_fetch<c1, B>(L, iblk, CH<real>);
        star_contract<N, false, Bv>(L, S, acc, [&](auto l0c, auto) {
            if constexpr (decltype(l0c)::value == 0) chunk_put<CH<real>>(L, r0);
            else chunk_put<c1>(L, r1);
        });
    } else {
        star_contract<N, false, Bv>(L, S, acc, [&](auto l0c, auto cntc) {
            constexpr int l0 = decltype(l0c)::value, cnt = decltype(cntc)::value;
            chunk_load<cnt, B>(L, iblk, l0);
        });
    }
}

template <int N, typename real>
__global__ void __launch_bounds__(64) k_volume(int64_t E, const real *__restrict__ I, const real *__restrict__ star,
                                               real *__restrict__ Q)
{
    constexpr int B = nb3(N);
    __shared__ real buf[NCOL * LB<real>];
    const Lane<real> L = make_lane(buf, E, logical_block());
    const Star<real> S = load_star(L, star);
    real acc[B];
#pragma unroll
    for (int k = 0; k < B; ++k) acc[k] = real(0);
    volume_acc<N>(L, S, I, acc, E);
    add_to_q<B>(L, Q, acc, E);
}

// tr += R^S^T rows [L0, L0+CNT) of a column staged in LDS (col[r] is row
// L0 + r), in ascending row order as face_trace.  In FP64 the chunk is one
// code block of its own: this keeps the per-stage flux kernels at two waves
// per SIMD (by the compiler's resource report), where eight-row blocks or no
// block boundary at all need more registers.
template <int N, int S, int L0, int CNT, typename real>
__device__ __forceinline__ void trace_rows(const real *col, real *tr)
{
    if (code_block<real>()) {
        static_for<0, CNT>([&](auto rj) {
            constexpr int r = decltype(rj)::value;
            RCol<N, S, L0 + r>::apply(col[r], tr);
        });
    }
    __builtin_amdgcn_sched_barrier(0);
}

// Local flux: Q += sum_S Rh^S (R^S^T I) A+^S^T   (per-stage form: the trace
// of each face is accumulated from I rows streamed through LDS)
template <int N, bool MIX, typename real>
__global__ void __launch_bounds__(64) k_local_flux(int64_t E, const real *__restrict__ I, const double *__restrict__ Ap,
                                                   real *__restrict__ Q)
{
    constexpr int B = nb3(N), Bf = nb2(N);
    __shared__ real buf[NCOL * LB<real>];
    const Lane<real> L = make_lane(buf, E, logical_block());
    real acc[B], tr[Bf];
#pragma unroll
    for (int k = 0; k < B; ++k) acc[k] = real(0);
    auto iblk = [&](int g) -> const real * { return I + slot_elem(L.base, g, E) * NQ * B; };
    static_for<0, 4>([&](auto si) {
        constexpr int S = decltype(si)::value;
#pragma unroll
        for (int m = 0; m < Bf; ++m) tr[m] = real(0);
        static_for<0, (B + CH<real> - 1) / CH<real>>([&](auto ci) {
            constexpr int l0 = decltype(ci)::value * CH<real>;
            constexpr int cnt = (B - l0) < CH<real> ? (B - l0) : CH<real>;
            chunk_load<cnt, B>(L, iblk, l0);
            lds_sync();
            trace_rows<N, S, l0, cnt>(L.own, tr);
            lds_sync();
        });
        flux_lift<N, S, MIX>(L, Ap + (L.elem * 4 + S) * 81, acc, [&](auto m0c, auto cntc) {
            constexpr int m0 = decltype(m0c)::value, cnt = decltype(cntc)::value;
            static_for<0, cnt>([&](auto ri) { L.own[ri] = tr[m0 + ri]; });
        });
    });
    add_to_q<B>(L, Q, acc, E);
}

// Neighbour flux: Q += sum_S Rh^S f^h (R^j^T I^nu) A-^S^T  (per-stage form)
template <int N, bool MIX, typename real>
__global__ void __launch_bounds__(64) k_neighbour_flux(int64_t E, int64_t nI, const real *__restrict__ I,
                                                       const int32_t *__restrict__ neigh,
                                                       const uint8_t *__restrict__ face_rot,
                                                       const double *__restrict__ Am, real *__restrict__ Q)
{
    constexpr int B = nb3(N), Bf = nb2(N);
    __shared__ real buf[NCOL * LB<real>];
    __shared__ int nbt[8][4];
    const Lane<real> L = make_lane(buf, E, logical_block());
    if (L.p == 0) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int nu = neigh[L.elem * 4 + s];
            nbt[L.e][s] = (nu >= 0 && nu < nI) ? nu : -1;   // out of range: no neighbour
        }
    }
    lds_sync();
    real acc[B], tr[Bf], t2[Bf];
#pragma unroll
    for (int k = 0; k < B; ++k) acc[k] = real(0);
    static_for<0, 4>([&](auto si) {
        constexpr int S = decltype(si)::value;
        const int nu = nbt[L.e][S];
        const uint8_t fr = face_rot[L.elem * 4 + S];
        const int j = fr & 3;
        // the neighbour's I streams through LDS in row chunks (zero rows when
        // there is no neighbour) and its face-j trace is accumulated per chunk
#pragma unroll
        for (int m = 0; m < Bf; ++m) tr[m] = real(0);
        static_for<0, (B + CH<real> - 1) / CH<real>>([&](auto ci) {
            constexpr int l0 = decltype(ci)::value * CH<real>;
            constexpr int cnt = (B - l0) < CH<real> ? (B - l0) : CH<real>;
            chunk_load<cnt, B>(L, [&](int g) -> const real * {
                const int n = nbt[g][S];
                return n >= 0 ? I + (int64_t)n * NQ * B : nullptr;
            }, l0);
            lds_sync();
            switch (j) {
            case 0: trace_rows<N, 0, l0, cnt>(L.own, tr); break;
            case 1: trace_rows<N, 1, l0, cnt>(L.own, tr); break;
            case 2: trace_rows<N, 2, l0, cnt>(L.own, tr); break;
            default: trace_rows<N, 3, l0, cnt>(L.own, tr); break;
            }
            lds_sync();
        });
        orient_rt<N>(fr >> 2, tr, t2);
        if (nu < 0) {
#pragma unroll
            for (int m = 0; m < Bf; ++m) t2[m] = real(0);
        }
        flux_lift<N, S, MIX>(L, Am + (L.elem * 4 + S) * 81, acc, [&](auto m0c, auto cntc) {
            constexpr int m0 = decltype(m0c)::value, cnt = decltype(cntc)::value;
            static_for<0, cnt>([&](auto ri) { L.own[ri] = t2[m0 + ri]; });
        });
    });
    add_to_q<B>(L, Q, acc, E);
}

// ---------------------------------------------------------------------------
// Time step.  One mesh of a step is described by a StepItem; the same device
// bodies serve a single mesh (one item) and a batch of meshes (a block-to-item
// table selects the item of each workgroup).
// ---------------------------------------------------------------------------
template <typename real>
struct StepItem {
    int64_t E;
    double dt;
    real *Q, *I, *traces;
    const real *star;
    const double *Ap, *Am;
    const int32_t *neigh;
    const uint8_t *face_rot;
    int64_t first_block;     // first workgroup of this item in a batched launch
    int64_t nI;              // neighbour index bound of the corrector (>= E)
};

// part 1: predictor + time integral (+ FP64 accumulation in the mixed form)
// + face traces of I;  part 2: volume + local flux + neighbour flux -> Q.
template <int N, bool MIX, typename real>
__global__ void __launch_bounds__(64)
k_step_predict(int64_t E, double dt, const real *__restrict__ Q, const real *__restrict__ star,
               real *__restrict__ Iout, real *__restrict__ traces)
{
    const int64_t lb = logical_block();
    __shared__ real buf[NCOL * LB<real>];
#include "step_predict_body.inc"
}

template <int N, bool MIX, typename real>
__global__ void __launch_bounds__(64)
k_step_correct(int64_t E, int64_t NI, const real *__restrict__ Iin, const real *__restrict__ traces,
               const real *__restrict__ star, const double *__restrict__ Ap, const double *__restrict__ Am,
               const int32_t *__restrict__ neigh, const uint8_t *__restrict__ face_rot, real *__restrict__ Q)
{
    const int64_t lb = logical_block();
    __shared__ real buf[NCOL * LB<real>];
#include "step_correct_body.inc"
}

// Fused step: the corrector of step n (reads I^n and the face traces of step
// n from tr_in, updates Q) followed, in the same workgroup, by the predictor
// of step n+1 on the updated Q (writes I^{n+1} over I^n and the traces of
// step n+1 to tr_out).  I is element local, so it is updated in place; the
// traces are read by neighbours and so go to the other buffer.  One launch per
// time step; Q^{n+1} is read back while still in cache.
template <int N, bool MIX, typename real>
__global__ void __launch_bounds__(64)
k_step_fused(int64_t E, double dt, real *__restrict__ I, const real *__restrict__ tr_in,
             real *__restrict__ tr_out, const real *__restrict__ star, const double *__restrict__ Ap,
             const double *__restrict__ Am, const int32_t *__restrict__ neigh,
             const uint8_t *__restrict__ face_rot, real *__restrict__ Q)
{
    const int64_t lb = logical_block();
    __shared__ real buf[NCOL * LB<real>];
    {
        const real *Iin = I, *traces = tr_in;
        const int64_t NI = E;
#include "step_correct_body.inc"
    }
    // this wave's stores of Q^{n+1} complete before it reads them back
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    lds_sync();
    // Opaque copies of the base pointers for the predictor, so that address
    // arithmetic of the corrector is not kept alive across both phases.  The
    // pointers escape into the asm and it clobbers memory, so the corrector's
    // stores of Q stay before it and the predictor's loads after it.
    real *Ip = I, *Qp = Q;
    const real *Sp = star;
    asm volatile("" : "+s"(Ip), "+s"(Qp), "+s"(Sp)::"memory");
    {
        const real *Q = Qp;
        const real *star = Sp;
        real *Iout = Ip;
        real *traces = tr_out;
#include "step_predict_body.inc"
    }
}

// Batched forms: every workgroup finds its item in block_item[] (items of one
// degree and precision, any number of meshes, one launch).
template <int N, bool MIX, typename real>
__global__ void __launch_bounds__(64)
k_batch_predict(const StepItem<real> *__restrict__ items,
                                                      const int32_t *__restrict__ block_item)
{
    const int64_t b = logical_block();
    const StepItem<real> &it = items[block_item[b]];
    const int64_t E = it.E, lb = b - it.first_block;
    const double dt = it.dt;
    const real *Q = it.Q, *star = it.star;
    real *Iout = it.I, *traces = it.traces;
    __shared__ real buf[NCOL * LB<real>];
#include "step_predict_body.inc"
}

template <int N, bool MIX, typename real>
__global__ void __launch_bounds__(64)
k_batch_correct(const StepItem<real> *__restrict__ items,
                                                      const int32_t *__restrict__ block_item)
{
    const int64_t b = logical_block();
    const StepItem<real> &it = items[block_item[b]];
    const int64_t E = it.E, NI = it.nI, lb = b - it.first_block;
    const real *Iin = it.I, *traces = it.traces, *star = it.star;
    const double *Ap = it.Ap, *Am = it.Am;
    const int32_t *neigh = it.neigh;
    const uint8_t *face_rot = it.face_rot;
    real *Q = it.Q;
    __shared__ real buf[NCOL * LB<real>];
#include "step_correct_body.inc"
}

// dense star [E][3][9][9] (FP64) -> packed [E][9][3][3] (real)
template <typename real>
__global__ void k_pack_star(int64_t E, const double *__restrict__ dense, real *__restrict__ packed)
{
    const int64_t n = E * 81;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = i / 81;
        const int r = i - e * 81, p = r / 9, d = (r % 9) / 3, s = r % 3;
        int q0, q1, q2;
        star_cols(p, q0, q1, q2);
        const int q = s == 0 ? q0 : (s == 1 ? q1 : q2);
        const bool pad = (s == 2) && (p >= 3 && p <= 5);
        packed[i] = pad ? real(0) : (real)dense[((e * 3 + d) * 9 + p) * 9 + q];
    }
}

}  // namespace dgk
