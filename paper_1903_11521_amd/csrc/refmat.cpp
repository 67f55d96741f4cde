// Reference matrices of the elastic ADER-DG scheme on the reference
// tetrahedron (paper Sec. 5.1: Dubiner basis, B = C(N+3,3) functions; the
// stiffness matrices of Sec. 2 Eq. stiffnesskernel; K-hat, K-tilde, R, R-hat
// and f with the shapes listed after Eq. seissol:correction_neigh).
//
// Method: collapsed-coordinate Gauss-Jacobi quadrature, nodes by Newton
// iteration with deflation on P_n^(a,0), weights 2^(a+1) / ((1-x^2) P_n'^2);
// basis functions and their gradients evaluated directly from the collapsed
// product form with the Jacobi derivative identity
// d/dx P_n^(a,b) = (n+a+b+1)/2 P_{n-1}^(a+1,b+1).  Masses use their closed
// forms.  Entries below 1e-13 * max|matrix| are set to exact 0.
//
// Conventions (fixed by this library's ABI):
//   phi_ijk = P_i(2xi/(1-eta-zeta)-1)(1-eta-zeta)^i P_j^(2i+1,0)(2eta/(1-zeta)-1)(1-zeta)^j
//             * P_k^(2i+2j+2,0)(2zeta-1);   order: degree d, then k, then j (i = d-j-k)
//   psi_ij  = P_i(2chi1/(1-chi2)-1)(1-chi2)^i P_j^(2i+1,0)(2chi2-1); order: d, then j
//   reference faces (vertex triples): (0,2,1) (0,1,3) (0,3,2) (1,2,3)
//   orientation h: chi -> (chi2,chi1) | (1-chi1-chi2,chi2) | (chi1,1-chi1-chi2)
#include "refmat.h"

#include <cmath>
#include <cstring>
#include <vector>

namespace dgref {

static double jacobi(int n, double a, double b, double x)
{
    if (n == 0) return 1.0;
    double p0 = 1.0, p1 = 0.5 * ((a + b + 2.0) * x + (a - b));
    for (int m = 2; m <= n; ++m) {
        double c = 2.0 * m + a + b;
        double a1 = 2.0 * m * (m + a + b) * (c - 2.0);
        double a2 = (c - 1.0) * (a * a - b * b);
        double a3 = (c - 2.0) * (c - 1.0) * c;
        double a4 = 2.0 * (m + a - 1.0) * (m + b - 1.0) * c;
        double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

static double djacobi(int n, double a, double b, double x)
{
    if (n == 0) return 0.0;
    return 0.5 * (n + a + b + 1.0) * jacobi(n - 1, a + 1.0, b + 1.0, x);
}

void gauss_jacobi(int n, double alpha, double *x, double *w)
{
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < n; ++k) {
        double r = -std::cos((2.0 * k + 1.0) * pi / (2.0 * n));
        if (k > 0) r = 0.5 * (r + x[k - 1]);
        for (int it = 0; it < 200; ++it) {
            double s = 0.0;
            for (int i = 0; i < k; ++i) s += 1.0 / (r - x[i]);
            double p = jacobi(n, alpha, 0.0, r);
            double dp = djacobi(n, alpha, 0.0, r);
            double delta = -p / (dp - s * p);
            r += delta;
            if (std::fabs(delta) < 1e-17) break;
        }
        x[k] = r;
    }
    for (int k = 0; k < n; ++k) {
        double dp = djacobi(n, alpha, 0.0, x[k]);
        w[k] = std::pow(2.0, alpha + 1.0) / ((1.0 - x[k] * x[k]) * dp * dp);
    }
}

struct Idx3 { int i, j, k; };
struct Idx2 { int i, j; };

static std::vector<Idx3> vol_indices(int N)
{
    std::vector<Idx3> v;
    for (int d = 0; d <= N; ++d)
        for (int k = 0; k <= d; ++k)
            for (int j = 0; j <= d - k; ++j) v.push_back({d - j - k, j, k});
    return v;
}

static std::vector<Idx2> face_indices(int N)
{
    std::vector<Idx2> v;
    for (int d = 0; d <= N; ++d)
        for (int j = 0; j <= d; ++j) v.push_back({d - j, j});
    return v;
}

// phi and its gradient at a point strictly inside the reference tetrahedron
static void eval_phi(const Idx3 &b, double xi, double eta, double zeta, double *val, double grad[3])
{
    const double s = 1.0 - eta - zeta, t = 1.0 - zeta;
    const double a = 2.0 * xi / s - 1.0, bb = 2.0 * eta / t - 1.0, c = 2.0 * zeta - 1.0;
    const int i = b.i, j = b.j, k = b.k;
    const double A = jacobi(i, 0, 0, a), dA = djacobi(i, 0, 0, a);
    const double Bv = jacobi(j, 2.0 * i + 1, 0, bb), dB = djacobi(j, 2.0 * i + 1, 0, bb);
    const double C = jacobi(k, 2.0 * i + 2 * j + 2, 0, c), dC = djacobi(k, 2.0 * i + 2 * j + 2, 0, c);
    const double si = std::pow(s, i), tj = std::pow(t, j);
    const double si1 = i > 0 ? std::pow(s, i - 1) : 0.0, tj1 = j > 0 ? std::pow(t, j - 1) : 0.0;
    const double F = A * si, G = Bv * tj;
    // dF/dxi = 2 A' s^{i-1};  dF/deta = dF/dzeta = s^{i-1} ((a+1) A' - i A)
    const double Fx = 2.0 * dA * (i > 0 ? si1 : 0.0);
    const double Fe = (i > 0) ? si1 * ((a + 1.0) * dA - i * A) : 0.0;
    // dG/deta = 2 B' t^{j-1};  dG/dzeta = t^{j-1} ((b+1) B' - j B)
    const double Ge = 2.0 * dB * (j > 0 ? tj1 : 0.0);
    const double Gz = (j > 0) ? tj1 * ((bb + 1.0) * dB - j * Bv) : 0.0;
    const double Hz = 2.0 * dC;
    *val = F * G * C;
    grad[0] = Fx * G * C;
    grad[1] = Fe * G * C + F * Ge * C;
    grad[2] = Fe * G * C + F * Gz * C + F * G * Hz;
}

static double eval_psi(const Idx2 &b, double c1, double c2)
{
    const double t = 1.0 - c2;
    const double a = (t > 0.0) ? 2.0 * c1 / t - 1.0 : -1.0;
    return jacobi(b.i, 0, 0, a) * std::pow(t, b.i) * jacobi(b.j, 2.0 * b.i + 1, 0, 2.0 * c2 - 1.0);
}

static const double REFV[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
static const int FACEV[4][3] = {{0, 2, 1}, {0, 1, 3}, {0, 3, 2}, {1, 2, 3}};

static void face_point(int s, double c1, double c2, double out[3])
{
    const double *a = REFV[FACEV[s][0]], *b = REFV[FACEV[s][1]], *c = REFV[FACEV[s][2]];
    for (int d = 0; d < 3; ++d) out[d] = a[d] + c1 * (b[d] - a[d]) + c2 * (c[d] - a[d]);
}

static void orient_point(int h, double c1, double c2, double *o1, double *o2)
{
    if (h == 0) { *o1 = c2; *o2 = c1; }
    else if (h == 1) { *o1 = 1.0 - c1 - c2; *o2 = c2; }
    else { *o1 = c1; *o2 = 1.0 - c1 - c2; }
}

static void snap(double *A, size_t n)
{
    double m = 0.0;
    for (size_t i = 0; i < n; ++i) m = std::fmax(m, std::fabs(A[i]));
    for (size_t i = 0; i < n; ++i)
        if (std::fabs(A[i]) < 1e-13 * m) A[i] = 0.0;
}

int basis_size(int N) { return (N + 1) * (N + 2) * (N + 3) / 6; }
int face_basis_size(int N) { return (N + 1) * (N + 2) / 2; }

size_t blob_size(int N)
{
    const size_t B = basis_size(N), F = face_basis_size(N);
    return 6 * B * B + 8 * B * F + 3 * F * F + B + F;
}

int build(int N, double *out)
{
    if (N < 1 || N > 8) return -1;
    const int B = basis_size(N), Bf = face_basis_size(N);
    const auto vi = vol_indices(N);
    const auto fi = face_indices(N);
    const int nq = N + 2;
    std::vector<double> x0(nq), w0(nq), x1(nq), w1(nq), x2(nq), w2(nq);
    gauss_jacobi(nq, 0.0, x0.data(), w0.data());
    gauss_jacobi(nq, 1.0, x1.data(), w1.data());
    gauss_jacobi(nq, 2.0, x2.data(), w2.data());

    std::vector<double> mass(B), fmass(Bf);
    for (int k = 0; k < B; ++k) {
        const Idx3 &b = vi[k];
        mass[k] = 1.0 / ((2.0 * b.i + 1) * (2.0 * b.i + 2 * b.j + 2) * (2.0 * b.i + 2 * b.j + 2 * b.k + 3));
    }
    for (int m = 0; m < Bf; ++m) fmass[m] = 1.0 / ((2.0 * fi[m].i + 1) * (2.0 * fi[m].i + 2 * fi[m].j + 2));

    // stiffness S^d_kl = int dphi_k/dxi_d phi_l
    std::vector<double> S(3 * (size_t)B * B, 0.0), val(B), grad(3 * (size_t)B);
    for (int a = 0; a < nq; ++a)
        for (int b = 0; b < nq; ++b)
            for (int c = 0; c < nq; ++c) {
                const double zeta = 0.5 * (1.0 + x2[c]);
                const double eta = 0.5 * (1.0 + x1[b]) * (1.0 - zeta);
                const double xi = 0.5 * (1.0 + x0[a]) * (1.0 - eta - zeta);
                const double w = w0[a] * w1[b] * w2[c] / 64.0;
                for (int k = 0; k < B; ++k) {
                    double g[3];
                    eval_phi(vi[k], xi, eta, zeta, &val[k], g);
                    for (int d = 0; d < 3; ++d) grad[d * B + k] = g[d];
                }
                for (int d = 0; d < 3; ++d)
                    for (int k = 0; k < B; ++k) {
                        const double gk = w * grad[d * B + k];
                        for (int l = 0; l < B; ++l) S[((size_t)d * B + k) * B + l] += gk * val[l];
                    }
            }
    double *Khat = out, *Ktil = Khat + 3 * (size_t)B * B, *R = Ktil + 3 * (size_t)B * B;
    double *Rhat = R + 4 * (size_t)B * Bf, *f = Rhat + 4 * (size_t)B * Bf;
    double *mout = f + 3 * (size_t)Bf * Bf, *fmout = mout + B;
    for (int d = 0; d < 3; ++d) {
        for (int k = 0; k < B; ++k)
            for (int l = 0; l < B; ++l) {
                Khat[((size_t)d * B + k) * B + l] = S[((size_t)d * B + k) * B + l] / mass[k];
                Ktil[((size_t)d * B + k) * B + l] = -S[((size_t)d * B + l) * B + k] / mass[k];
            }
        snap(Khat + (size_t)d * B * B, (size_t)B * B);
        snap(Ktil + (size_t)d * B * B, (size_t)B * B);
    }
    // face matrices on the reference triangle (collapsed rule, weight sum 1/2)
    std::vector<double> psi(Bf), phis(B);
    for (int s = 0; s < 4; ++s) {
        std::vector<double> raw((size_t)B * Bf, 0.0);
        for (int a = 0; a < nq; ++a)
            for (int b = 0; b < nq; ++b) {
                const double c2 = 0.5 * (1.0 + x1[b]);
                const double c1 = 0.5 * (1.0 + x0[a]) * (1.0 - c2);
                const double w = w0[a] * w1[b] / 8.0;
                double p[3];
                face_point(s, c1, c2, p);
                for (int m = 0; m < Bf; ++m) psi[m] = eval_psi(fi[m], c1, c2);
                for (int l = 0; l < B; ++l) {
                    double g[3];
                    eval_phi(vi[l], p[0], p[1], p[2], &phis[l], g);
                }
                for (int l = 0; l < B; ++l)
                    for (int m = 0; m < Bf; ++m) raw[(size_t)l * Bf + m] += w * phis[l] * psi[m];
            }
        for (int l = 0; l < B; ++l)
            for (int m = 0; m < Bf; ++m) {
                R[((size_t)s * B + l) * Bf + m] = raw[(size_t)l * Bf + m] / fmass[m];
                Rhat[((size_t)s * B + l) * Bf + m] = raw[(size_t)l * Bf + m] / mass[l];
            }
        snap(R + (size_t)s * B * Bf, (size_t)B * Bf);
        snap(Rhat + (size_t)s * B * Bf, (size_t)B * Bf);
    }
    for (int h = 0; h < 3; ++h) {
        std::vector<double> raw((size_t)Bf * Bf, 0.0), psih(Bf);
        for (int a = 0; a < nq; ++a)
            for (int b = 0; b < nq; ++b) {
                const double c2 = 0.5 * (1.0 + x1[b]);
                const double c1 = 0.5 * (1.0 + x0[a]) * (1.0 - c2);
                const double w = w0[a] * w1[b] / 8.0;
                double o1, o2;
                orient_point(h, c1, c2, &o1, &o2);
                for (int m = 0; m < Bf; ++m) {
                    psi[m] = eval_psi(fi[m], c1, c2);
                    psih[m] = eval_psi(fi[m], o1, o2);
                }
                for (int m = 0; m < Bf; ++m)
                    for (int n = 0; n < Bf; ++n) raw[(size_t)m * Bf + n] += w * psi[m] * psih[n];
            }
        for (int m = 0; m < Bf; ++m)
            for (int n = 0; n < Bf; ++n) f[((size_t)h * Bf + m) * Bf + n] = raw[(size_t)m * Bf + n] / fmass[m];
        snap(f + (size_t)h * Bf * Bf, (size_t)Bf * Bf);
    }
    std::memcpy(mout, mass.data(), sizeof(double) * B);
    std::memcpy(fmout, fmass.data(), sizeof(double) * Bf);
    return 0;
}

}  // namespace dgref

#ifdef DG_REFMAT_STANDALONE
// C entry points of a host-only build of this file (used by the build-time
// code generator before the HIP library exists).
#include <cstdint>
extern "C" int64_t dg_reference_blob_size(int degree)
{
    return (degree < 1 || degree > 8) ? -1 : (int64_t)dgref::blob_size(degree);
}
extern "C" int dg_reference_matrices(int degree, double *out)
{
    return (out && degree >= 1 && degree <= 8 && dgref::build(degree, out) == 0) ? 0 : -1;
}
#endif
