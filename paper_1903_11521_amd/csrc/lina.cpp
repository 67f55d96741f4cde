// Host part of the LinA ADER-DG-SEM scheme (Sec. 5.2): the coefficient blob
// (Gauss-Lobatto nodes and weights, the collocation derivative matrices,
// acoustic star matrices and side flux solvers) and the C ABI of the step.
#include "dg.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "dg_internal.h"
#include "lina_internal.h"

namespace {

int fail(int code, const char *fmt, long long a = 0, long long b = 0)
{
    char buf[512];
    std::snprintf(buf, sizeof buf, fmt, a, b);
    return dg_set_error(code, buf);
}

// Legendre P_n and P_n' at x by the three-term recurrence.
void legendre(int n, double x, double &p, double &dp)
{
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (n == 0) {
        p = 1.0, dp = 0.0;
        return;
    }
    for (int k = 2; k <= n; ++k) {
        const double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        const double d2 = d0 + (2 * k - 1) * p1;   // P_k' = P_{k-2}' + (2k-1) P_{k-1}
        p0 = p1, p1 = p2, d0 = d1, d1 = d2;
    }
    p = p1, dp = d1;
}

}  // namespace

int lina_blob(int O, double rho0, double K0, double h, double *out)
{
    const int N = O - 1;
    std::vector<double> x((size_t)O), w((size_t)O);
    // nodes on [-1, 1]: the endpoints and the roots of P_N', by Newton from
    // the Chebyshev-Gauss-Lobatto points, using (1 - x^2) P_N'' = 2 x P_N' - N (N+1) P_N
    x[0] = -1.0, x[(size_t)N] = 1.0;
    for (int j = 1; j < N; ++j) {
        double t = -std::cos(M_PI * j / N);
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(N, t, p, dp);
            const double d2 = (2.0 * t * dp - N * (N + 1.0) * p) / (1.0 - t * t);
            const double step = dp / d2;
            t -= step;
            if (std::fabs(step) < 1e-16) break;
        }
        x[(size_t)j] = t;
    }
    std::vector<double> P((size_t)O);
    for (int j = 0; j < O; ++j) {
        double p, dp;
        legendre(N, x[(size_t)j], p, dp);
        P[(size_t)j] = p;
        w[(size_t)j] = 1.0 / (N * (N + 1.0) * p * p);   // 2/(N(N+1)P^2) on [-1,1], halved for [0,1]
    }
    // collocation derivative on [0, 1] (twice the [-1, 1] one):
    // D_ij = P_N(x_i) / (P_N(x_j) (x_i - x_j)), D_00 = -N(N+1)/4, D_NN = N(N+1)/4
    double *Kt = out, *Kh = out + O * O, *wo = out + 2 * O * O, *star = wo + O, *Ap = star + 48, *Am = Ap + 96;
    std::vector<double> D((size_t)O * O, 0.0);
    for (int i = 0; i < O; ++i)
        for (int j = 0; j < O; ++j)
            if (i != j) D[(size_t)(i * O + j)] = 2.0 * P[(size_t)i] / (P[(size_t)j] * (x[(size_t)i] - x[(size_t)j]));
    D[0] = -N * (N + 1.0) / 2.0;
    D[(size_t)(O * O - 1)] = N * (N + 1.0) / 2.0;
    for (int i = 0; i < O; ++i)
        for (int j = 0; j < O; ++j) {
            Kt[i * O + j] = -D[(size_t)(i * O + j)];
            Kh[i * O + j] = w[(size_t)j] / w[(size_t)i] * D[(size_t)(j * O + i)];
        }
    for (int i = 0; i < O; ++i) wo[i] = w[(size_t)i];
    // acoustic Jacobians J_d: (p row, u_d column) = K0, (u_d row, p column) = 1/rho0
    const double c = std::sqrt(K0 / rho0);
    for (int i = 0; i < 48 + 192; ++i) star[i] = 0.0;
    for (int d = 0; d < 3; ++d) {
        star[d * 16 + 0 * 4 + (1 + d)] = K0 / h;
        star[d * 16 + (1 + d) * 4 + 0] = 1.0 / (rho0 * h);
    }
    for (int s = 0; s < 6; ++s) {
        const int d = s / 2;
        const double sg = s % 2 ? 1.0 : -1.0;      // outward normal -e_d or +e_d
        double *ap = Ap + s * 16, *am = Am + s * 16;
        // A_n = sg J_d; |A_n| = c on p and u_d
        const double jpu = sg * K0, jup = sg / rho0;
        ap[0 * 4 + 0] = -c / (2 * h), am[0 * 4 + 0] = c / (2 * h);
        ap[(1 + d) * 4 + (1 + d)] = -c / (2 * h), am[(1 + d) * 4 + (1 + d)] = c / (2 * h);
        ap[0 * 4 + (1 + d)] = -jpu / (2 * h), am[0 * 4 + (1 + d)] = -jpu / (2 * h);
        ap[(1 + d) * 4 + 0] = -jup / (2 * h), am[(1 + d) * 4 + 0] = -jup / (2 * h);
    }
    return 0;
}

extern "C" {

int64_t dg_lina_blob_size(int order)
{
    if (order < 2 || order > DG_LINA_MAX_ORDER_FP32) return -1;
    return 2 * (int64_t)order * order + order + 48 + 192;
}

int dg_lina_coefficients(int order, double rho0, double K0, double h, double *out)
{
    if (order < 2 || order > DG_LINA_MAX_ORDER_FP32)
        return fail(DG_EUNSUPPORTED, "dg_lina_coefficients: order %lld outside [2, %lld]", order,
                    DG_LINA_MAX_ORDER_FP32);
    if (!out) return fail(DG_EINVAL, "dg_lina_coefficients: null output");
    if (!(rho0 > 0.0) || !(K0 > 0.0) || !(h > 0.0) || !std::isfinite(rho0 * K0 * h))
        return fail(DG_EINVAL, "dg_lina_coefficients: rho0, K0 and h must be positive and finite");
    lina_blob(order, rho0, K0, h, out);
    return DG_OK;
}

int dg_lina_step(dg_precision precision, int order, int64_t E, int n_steps, double dt, void *Q, void *sides,
                 const double *coef, const int32_t *neigh, hipStream_t stream)
{
    if (precision != DG_FP64 && precision != DG_FP32)
        return fail(DG_EUNSUPPORTED, "dg_lina_step: precision %lld is neither DG_FP64 nor DG_FP32", precision);
    const int omax = precision == DG_FP64 ? DG_LINA_MAX_ORDER_FP64 : DG_LINA_MAX_ORDER_FP32;
    if (order < 2 || order > omax)
        return fail(DG_EUNSUPPORTED, "dg_lina_step: order %lld outside [2, %lld] for this precision", order, omax);
    if (E < 0 || E > 0x7fffffff) return fail(DG_EINVAL, "dg_lina_step: element count %lld out of range", E);
    if (n_steps < 0) return fail(DG_EINVAL, "dg_lina_step: negative step count %lld", n_steps);
    if (E == 0 || n_steps == 0) return DG_OK;
    if (!Q || !sides || !coef || !neigh) return fail(DG_EINVAL, "dg_lina_step: null pointer");
    if (!std::isfinite(dt)) return fail(DG_EINVAL, "dg_lina_step: dt not finite");
    for (int s = 0; s < n_steps; ++s) {
        hipError_t e = lina_launch(precision == DG_FP64, order, E, dt, Q, sides, coef, neigh, stream);
        if (e != hipSuccess) {
            char buf[256];
            std::snprintf(buf, sizeof buf, "dg_lina_step: HIP error %d (%s)", (int)e, hipGetErrorString(e));
            return dg_set_error(DG_EHIP, buf);
        }
    }
    return DG_OK;
}

}  // extern "C"
