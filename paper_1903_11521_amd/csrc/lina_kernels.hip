// Kernels of the LinA ADER-DG-SEM scheme (Sec. 5.2) for linear acoustics on
// a uniform periodic grid of cubes with a tensor-product Gauss-Lobatto
// nodal basis of order O (degree N = O - 1).  Q [E][4][O][O][O] with x
// fastest (quantities p, u, v, w); sides [E][6][4][O][O] in the order left,
// right, bottom, top, back, front, each over the two remaining directions
// (z, y), (z, x) or (y, x); neigh [E][6] in the same side order.
//
// k_lina_predict (one workgroup per element): the derivatives of Eq.
// lina:derivative with the acoustic star matrices (A*, B*, C* couple p with
// u, v, w), the time integral of Eq. lina:integration, the side values of
// Eq. lin3d_evaluateSide, and Q* = Q + the weak derivatives.  The element's
// derivative lives in five LDS buffers of O^2 (O+1) values (x rows padded to
// O+1): p (two, current and next), u, v, w, as Taylor-scaled derivatives
// T^d = dt^d/d! D^d.  One derivative is three line passes (s = dt/(d+1)):
// the x pass reads the x-lines of p and u, writes p_next = s a_x Kt u and
// u = s b_x Kt p; the y pass adds s a_y Kt v to p_next and writes
// v = s b_y Kt p; the z pass likewise with w.  A thread owns one line per
// direction and accumulates the time integral of the values it reads in
// registers.  k_lina_flux (one workgroup per element) adds the side fluxes
// of Eq. lina3d_flux to the boundary nodes, one direction at a time.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lina_internal.h"

namespace dgn {

template <int O>
constexpr int threads() { return ((O * O + 63) / 64) * 64; }

template <int O>
constexpr int lds_values() { return 5 * O * O * (O + 1); }

template <typename real>
struct Coef {
    const real *Kt, *Kh, *w, *star, *Ap, *Am;
};

template <typename real, int O>
__device__ __forceinline__ Coef<real> coef_of(const real *c)
{
    Coef<real> k;
    k.Kt = c;
    k.Kh = c + O * O;
    k.w = c + 2 * O * O;
    k.star = k.w + O;
    k.Ap = k.star + 48;
    k.Am = k.Ap + 96;
    return k;
}

// out[x] = sum_l K[x][l] in[l], scaled
template <typename real, int O>
__device__ __forceinline__ void line_apply(const real *__restrict__ K, const real (&in)[O], real (&out)[O], real s)
{
#pragma unroll
    for (int x = 0; x < O; ++x) {
        real a = real(0);
#pragma unroll
        for (int l = 0; l < O; ++l) a = fma(K[x * O + l], in[l], a);
        out[x] = s * a;
    }
}

template <typename real, int O>
__global__ void __launch_bounds__(threads<O>())
k_lina_predict(double dt, real *__restrict__ Q, real *__restrict__ sides, const real *__restrict__ coef)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    constexpr int N = O - 1, S = O + 1, O2 = O * O, O3 = O2 * O, BUF = O2 * S, T = threads<O>();
    real *buf = reinterpret_cast<real *>(lds_raw);
    real *bp[2] = {buf, buf + BUF};
    real *bu = buf + 2 * BUF, *bv = buf + 3 * BUF, *bw = buf + 4 * BUF;
    const Coef<real> k = coef_of<real, O>(coef);
    const real ax = k.star[0 * 16 + 1], bx = k.star[0 * 16 + 4];
    const real ay = k.star[1 * 16 + 2], by = k.star[1 * 16 + 8];
    const real az = k.star[2 * 16 + 3], bz = k.star[2 * 16 + 12];
    const int t = threadIdx.x;
    const int64_t e = blockIdx.x;
    real *Qe = Q + e * 4 * O3;
    auto lidx = [](int x, int y, int z) { return (z * O + y) * S + x; };
    // load Q into the p, u, v, w buffers
    for (int i = t; i < 4 * O3; i += T) {
        const int q = i / O3, r = i - q * O3, x = r % O, y = (r / O) % O, z = r / O2;
        real *dst = q == 0 ? bp[0] : q == 1 ? bu : q == 2 ? bv : bw;
        dst[lidx(x, y, z)] = Qe[i];
    }
    // line owned in each direction: x-line (y, z), y-line (x, z), z-line (x, y)
    const bool own = t < O2;
    const int la = t % O, lb = t / O;
    real Ip[O], Iu[O], Iv[O], Iw[O];
#pragma unroll
    for (int i = 0; i < O; ++i) Ip[i] = Iu[i] = Iv[i] = Iw[i] = real(0);
    // The buffers carry Taylor-scaled derivatives T^d = dt^d/d! D^d (the
    // unscaled ones of rough data leave the FP32 range by d = 7 at order 16):
    // T^(d+1) = dt/(d+1) * (the derivative of T^d), I = sum_d dt/(d+1) T^d.
    int cur = 0;
    for (int d = 0; d <= N; ++d) {
        const real cd = (real)(dt / (d + 1));
        const real sx = cd * ax, tx = cd * bx, sy = cd * ay, ty = cd * by, sz = cd * az, tz = cd * bz;
        const bool last = d == N;    // accumulate T^N only
        real *pc = bp[cur], *pn = bp[cur ^ 1];
        __syncthreads();
        if (own) {      // x pass: p and u along x at (y, z) = (la, lb)
            real pl[O], ul[O], o1[O], o2[O];
#pragma unroll
            for (int i = 0; i < O; ++i) pl[i] = pc[lidx(i, la, lb)], ul[i] = bu[lidx(i, la, lb)];
#pragma unroll
            for (int i = 0; i < O; ++i) Ip[i] = fma(cd, pl[i], Ip[i]), Iu[i] = fma(cd, ul[i], Iu[i]);
            if (!last) {
                line_apply<real, O>(k.Kt, ul, o1, sx);
                line_apply<real, O>(k.Kt, pl, o2, tx);
#pragma unroll
                for (int i = 0; i < O; ++i) pn[lidx(i, la, lb)] = o1[i], bu[lidx(i, la, lb)] = o2[i];
            }
        }
        __syncthreads();
        if (own) {      // y pass at (x, z) = (la, lb)
            real pl[O], vl[O], o1[O], o2[O];
#pragma unroll
            for (int i = 0; i < O; ++i) pl[i] = pc[lidx(la, i, lb)], vl[i] = bv[lidx(la, i, lb)];
#pragma unroll
            for (int i = 0; i < O; ++i) Iv[i] = fma(cd, vl[i], Iv[i]);
            if (!last) {
                line_apply<real, O>(k.Kt, vl, o1, sy);
                line_apply<real, O>(k.Kt, pl, o2, ty);
#pragma unroll
                for (int i = 0; i < O; ++i) pn[lidx(la, i, lb)] += o1[i], bv[lidx(la, i, lb)] = o2[i];
            }
        }
        __syncthreads();
        if (own) {      // z pass at (x, y) = (la, lb)
            real pl[O], wl[O], o1[O], o2[O];
#pragma unroll
            for (int i = 0; i < O; ++i) pl[i] = pc[lidx(la, lb, i)], wl[i] = bw[lidx(la, lb, i)];
#pragma unroll
            for (int i = 0; i < O; ++i) Iw[i] = fma(cd, wl[i], Iw[i]);
            if (!last) {
                line_apply<real, O>(k.Kt, wl, o1, sz);
                line_apply<real, O>(k.Kt, pl, o2, tz);
#pragma unroll
                for (int i = 0; i < O; ++i) pn[lidx(la, lb, i)] += o1[i], bw[lidx(la, lb, i)] = o2[i];
            }
        }
        cur ^= 1;
    }
    // the time integral into LDS: p in bp[0], u, v, w in their buffers;
    // bp[1] receives the weak derivative of p
    __syncthreads();
    real *ip = bp[0], *dp = bp[1];
    if (own) {
#pragma unroll
        for (int i = 0; i < O; ++i) {
            ip[lidx(i, la, lb)] = Ip[i];
            bu[lidx(i, la, lb)] = Iu[i];
            bv[lidx(la, i, lb)] = Iv[i];
            bw[lidx(la, lb, i)] = Iw[i];
        }
    }
    __syncthreads();
    // sides of I (Eq. lin3d_evaluateSide)
    real *Xe = sides + e * 6 * 4 * O2;
    for (int i = t; i < 6 * 4 * O2; i += T) {
        const int s = i / (4 * O2), r = i - s * 4 * O2, q = r / O2, ab = r - q * O2, a = ab / O, b = ab % O;
        const int edge = (s & 1) ? N : 0;
        const real *src = q == 0 ? ip : q == 1 ? bu : q == 2 ? bv : bw;
        const int li = s < 2 ? lidx(edge, b, a) : s < 4 ? lidx(b, edge, a) : lidx(b, a, edge);
        Xe[i] = src[li];
    }
    __syncthreads();
    // weak derivatives: dp = sum_d a_d Kh_d I_(u,v,w); u, v, w = b_d Kh_d I_p
    if (own) {
        real pl[O], ul[O], o1[O], o2[O];
#pragma unroll
        for (int i = 0; i < O; ++i) pl[i] = ip[lidx(i, la, lb)], ul[i] = bu[lidx(i, la, lb)];
        line_apply<real, O>(k.Kh, ul, o1, ax);
        line_apply<real, O>(k.Kh, pl, o2, bx);
#pragma unroll
        for (int i = 0; i < O; ++i) dp[lidx(i, la, lb)] = o1[i], bu[lidx(i, la, lb)] = o2[i];
    }
    __syncthreads();
    if (own) {
        real pl[O], vl[O], o1[O], o2[O];
#pragma unroll
        for (int i = 0; i < O; ++i) pl[i] = ip[lidx(la, i, lb)], vl[i] = bv[lidx(la, i, lb)];
        line_apply<real, O>(k.Kh, vl, o1, ay);
        line_apply<real, O>(k.Kh, pl, o2, by);
#pragma unroll
        for (int i = 0; i < O; ++i) dp[lidx(la, i, lb)] += o1[i], bv[lidx(la, i, lb)] = o2[i];
    }
    __syncthreads();
    if (own) {
        real pl[O], wl[O], o1[O], o2[O];
#pragma unroll
        for (int i = 0; i < O; ++i) pl[i] = ip[lidx(la, lb, i)], wl[i] = bw[lidx(la, lb, i)];
        line_apply<real, O>(k.Kh, wl, o1, az);
        line_apply<real, O>(k.Kh, pl, o2, bz);
#pragma unroll
        for (int i = 0; i < O; ++i) dp[lidx(la, lb, i)] += o1[i], bw[lidx(la, lb, i)] = o2[i];
    }
    __syncthreads();
    // Q* = Q + weak derivatives
    for (int i = t; i < 4 * O3; i += T) {
        const int q = i / O3, r = i - q * O3, x = r % O, y = (r / O) % O, z = r / O2;
        const real *src = q == 0 ? dp : q == 1 ? bu : q == 2 ? bv : bw;
        Qe[i] += src[lidx(x, y, z)];
    }
}

// Eq. lina3d_flux: Q += Fh (X_own Ap^T + X_neigh Am^T) on the nodes of each
// side, one direction at a time (edge and corner nodes belong to several).
template <typename real, int O>
__global__ void __launch_bounds__(threads<O>())
k_lina_flux(int64_t E, real *__restrict__ Q, const real *__restrict__ sides, const real *__restrict__ coef,
            const int32_t *__restrict__ neigh)
{
    constexpr int N = O - 1, O2 = O * O, O3 = O2 * O;
    const Coef<real> k = coef_of<real, O>(coef);
    const int t = threadIdx.x;
    const int64_t e = blockIdx.x;
    real *Qe = Q + e * 4 * O3;
    const int a = t / O, b = t % O;
    for (int d = 0; d < 3; ++d) {
        if (t < O2) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int s = 2 * d + h, edge = h ? N : 0;
                const int64_t nb = neigh[e * 6 + s];
                const bool has = nb >= 0 && nb < E;      // out of range: no neighbour term
                const real *xo = sides + (e * 6 + s) * 4 * O2 + a * O + b;
                const real *xn = sides + ((has ? nb : e) * 6 + (s ^ 1)) * 4 * O2 + a * O + b;
                real vo[4], vn[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) vo[q] = xo[q * O2], vn[q] = has ? xn[q * O2] : real(0);
                const int node = d == 0 ? (a * O + b) * O + edge : d == 1 ? (a * O + edge) * O + b : (edge * O + a) * O + b;
                const real inv = real(1) / k.w[edge];
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    real g = real(0);
#pragma unroll
                    for (int q = 0; q < 4; ++q) g = fma(k.Ap[s * 16 + p * 4 + q], vo[q], fma(k.Am[s * 16 + p * 4 + q], vn[q], g));
                    Qe[p * O3 + node] += inv * g;
                }
            }
        }
        __syncthreads();
    }
}

template <typename real, int O>
hipError_t launch(int64_t E, double dt, void *Q, void *sides, const void *coef, const int32_t *neigh, hipStream_t s)
{
    const size_t lds = (size_t)lds_values<O>() * sizeof(real);
    static bool attr = false;     // the dynamic LDS limit, set once per instantiation
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)k_lina_predict<real, O>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((k_lina_predict<real, O>), dim3((unsigned)E), dim3(threads<O>()), lds, s, dt, (real *)Q,
                       (real *)sides, (const real *)coef);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_lina_flux<real, O>), dim3((unsigned)E), dim3(threads<O>()), 0, s, E, (real *)Q,
                       (const real *)sides, (const real *)coef, neigh);
    return hipGetLastError();
}

template <typename real, int O>
struct Dispatch {
    static hipError_t run(int o, int64_t E, double dt, void *Q, void *sides, const void *coef, const int32_t *neigh,
                          hipStream_t s)
    {
        if (o == O) return launch<real, O>(E, dt, Q, sides, coef, neigh, s);
        return Dispatch<real, O - 1>::run(o, E, dt, Q, sides, coef, neigh, s);
    }
};
template <typename real>
struct Dispatch<real, 1> {
    static hipError_t run(int, int64_t, double, void *, void *, const void *, const int32_t *, hipStream_t)
    {
        return hipErrorInvalidValue;
    }
};

}  // namespace dgn

hipError_t lina_launch(bool fp64, int O, int64_t E, double dt, void *Q, void *sides, const void *coef,
                       const int32_t *neigh, hipStream_t s)
{
    if (fp64) return dgn::Dispatch<double, 12>::run(O, E, dt, Q, sides, coef, neigh, s);
    return dgn::Dispatch<float, 16>::run(O, E, dt, Q, sides, coef, neigh, s);
}
