// Per-element static data of the elastic ADER-DG scheme (host code, FP64).
//
// * Star matrices (paper Sec. 5.1.1: element-dependent linear combinations
//   of the Jacobians A, B, C of Eq. linearpde):  A*^d = sum_j G_dj A^(j),
//   G = J^-1, J = [x1-x0 | x2-x0 | x3-x0].
// * Flux-solver matrices A+ / A- (Sec. 5.1.1, "solution to the 1D Riemann
//   problem" on each face).  Reading: exact Godunov flux between two
//   isotropic elastic materials.  In the face frame (normal n, tangents s,
//   t) the left-going P and S waves carry the amplitudes
//     u_P = (d_nn + Zp_R d_un) / (Zp_L + Zp_R),
//     u_S = (d_ns + Zs_R d_us) / (Zs_L + Zs_R)   (same for t),
//   d = q_R - q_L, Z = rho c; the interface flux is A_L q_L + W d with
//   W = -(r_P u_P + r_S1 u_S1 + r_S2 u_S2), r_P = (l+2m, l, l, 0,0,0, cp,0,0),
//   r_S1 = m e_ns + cs e_vs, r_S2 = m e_nt + cs e_wt.  Then
//   A+ = -(2|S|/det J) T (A_L - W) T^-1,  A- = -(2|S|/det J) T W T^-1,
//   T the 9x9 rotation face frame -> global (velocity Q v, stress Q s Q^T).
// Quantity order: s_xx s_yy s_zz s_xy s_yz s_xz u v w.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

const int FACEV[4][3] = {{0, 2, 1}, {0, 1, 3}, {0, 3, 2}, {1, 2, 3}};
const int VOIGT[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {1, 2}, {0, 2}};

struct Mat { double rho, lam, mu, cp, cs; };

Mat material(const double *m)
{
    Mat r;
    r.rho = m[0];
    r.cp = m[1];
    r.cs = m[2];
    r.mu = r.rho * r.cs * r.cs;
    r.lam = r.rho * r.cp * r.cp - 2.0 * r.mu;
    return r;
}

// Jacobian of direction j (0=x,1=y,2=z), dense 9x9 row-major, added with weight g
void add_jacobian(double *A, int j, const Mat &m, double g)
{
    const double l2m = m.lam + 2.0 * m.mu, ir = 1.0 / m.rho;
    auto set = [&](int r, int c, double v) { A[r * 9 + c] += g * v; };
    if (j == 0) {
        set(0, 6, -l2m); set(1, 6, -m.lam); set(2, 6, -m.lam); set(3, 7, -m.mu); set(5, 8, -m.mu);
        set(6, 0, -ir); set(7, 3, -ir); set(8, 5, -ir);
    } else if (j == 1) {
        set(0, 7, -m.lam); set(1, 7, -l2m); set(2, 7, -m.lam); set(3, 6, -m.mu); set(4, 8, -m.mu);
        set(6, 3, -ir); set(7, 1, -ir); set(8, 4, -ir);
    } else {
        set(0, 8, -m.lam); set(1, 8, -m.lam); set(2, 8, -l2m); set(4, 7, -m.mu); set(5, 6, -m.mu);
        set(6, 5, -ir); set(7, 4, -ir); set(8, 2, -ir);
    }
}

void rotation(const double Qm[3][3], double T[81])
{
    // Qm[a][i]: component a of frame vector i (columns n, s, t)
    std::memset(T, 0, sizeof(double) * 81);
    for (int col = 0; col < 6; ++col) {
        const int i = VOIGT[col][0], j = VOIGT[col][1];
        for (int row = 0; row < 6; ++row) {
            const int a = VOIGT[row][0], b = VOIGT[row][1];
            double v = Qm[a][i] * Qm[b][j];
            if (i != j) v += Qm[a][j] * Qm[b][i];
            T[row * 9 + col] = v;
        }
    }
    for (int a = 0; a < 3; ++a)
        for (int i = 0; i < 3; ++i) T[(6 + a) * 9 + 6 + i] = Qm[a][i];
}

void matmul9(const double *A, const double *B, double *C)
{
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 9; ++j) {
            double s = 0.0;
            for (int k = 0; k < 9; ++k) s += A[i * 9 + k] * B[k * 9 + j];
            C[i * 9 + j] = s;
        }
}

void one_element(int64_t e, const double *X, const double *mats, const int32_t *neigh,
                 double *star, double *Ap, double *Am)
{
    const double *x = X + e * 12;
    double J[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) J[r][c] = x[(c + 1) * 3 + r] - x[r];
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
                     - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
                     + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    double G[3][3];
    G[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    G[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    G[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    G[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    G[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    G[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    G[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    G[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    G[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    const Mat mL = material(mats + e * 3);
    double *st = star + e * 243;
    std::memset(st, 0, sizeof(double) * 243);
    for (int d = 0; d < 3; ++d)
        for (int j = 0; j < 3; ++j) add_jacobian(st + d * 81, j, mL, G[d][j]);

    for (int s = 0; s < 4; ++s) {
        const double *a = x + FACEV[s][0] * 3, *b = x + FACEV[s][1] * 3, *c = x + FACEV[s][2] * 3;
        double ab[3], ac[3], cr[3];
        for (int k = 0; k < 3; ++k) { ab[k] = b[k] - a[k]; ac[k] = c[k] - a[k]; }
        cr[0] = ab[1] * ac[2] - ab[2] * ac[1];
        cr[1] = ab[2] * ac[0] - ab[0] * ac[2];
        cr[2] = ab[0] * ac[1] - ab[1] * ac[0];
        const double ncr = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        const double nab = std::sqrt(ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2]);
        double n[3], sv[3], t[3];
        for (int k = 0; k < 3; ++k) { n[k] = cr[k] / ncr; sv[k] = ab[k] / nab; }
        t[0] = n[1] * sv[2] - n[2] * sv[1];
        t[1] = n[2] * sv[0] - n[0] * sv[2];
        t[2] = n[0] * sv[1] - n[1] * sv[0];
        double Qm[3][3], Qt[3][3];
        for (int k = 0; k < 3; ++k) {
            Qm[k][0] = n[k]; Qm[k][1] = sv[k]; Qm[k][2] = t[k];
        }
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) Qt[r][q] = Qm[q][r];
        double T[81], Ti[81];
        rotation(Qm, T);
        rotation(Qt, Ti);
        const int32_t nb = neigh[e * 4 + s];
        const Mat mR = material(mats + (nb >= 0 ? (int64_t)nb : e) * 3);
        const double ZpL = mL.rho * mL.cp, ZpR = mR.rho * mR.cp;
        const double ZsL = mL.rho * mL.cs, ZsR = mR.rho * mR.cs;
        double W[81] = {0}, AL[81] = {0};
        add_jacobian(AL, 0, mL, 1.0);
        const double rP[9] = {mL.lam + 2 * mL.mu, mL.lam, mL.lam, 0, 0, 0, mL.cp, 0, 0};
        const double iP = 1.0 / (ZpL + ZpR), iS = 1.0 / (ZsL + ZsR);
        for (int r = 0; r < 9; ++r) {
            W[r * 9 + 0] -= rP[r] * iP;
            W[r * 9 + 6] -= rP[r] * ZpR * iP;
        }
        W[3 * 9 + 3] -= mL.mu * iS; W[3 * 9 + 7] -= mL.mu * ZsR * iS;
        W[7 * 9 + 3] -= mL.cs * iS; W[7 * 9 + 7] -= mL.cs * ZsR * iS;
        W[5 * 9 + 5] -= mL.mu * iS; W[5 * 9 + 8] -= mL.mu * ZsR * iS;
        W[8 * 9 + 5] -= mL.cs * iS; W[8 * 9 + 8] -= mL.cs * ZsR * iS;
        double Pp[81], Pm[81], tmp[81];
        for (int k = 0; k < 81; ++k) Pp[k] = AL[k] - W[k];
        const double scale = -(ncr) / det;   // -(2|S|/det J), |S| = ncr/2
        double *outp = Ap + (e * 4 + s) * 81, *outm = Am + (e * 4 + s) * 81;
        matmul9(T, Pp, tmp);
        matmul9(tmp, Ti, outp);
        matmul9(T, W, tmp);
        matmul9(tmp, Ti, Pm);
        for (int k = 0; k < 81; ++k) {
            outp[k] *= scale;
            outm[k] = nb >= 0 ? scale * Pm[k] : 0.0;
        }
    }
}

// Viscoelastic element (three mechanisms): star [3][27][9] and flux solvers
// [4][27][9] acting on the 9 elastic columns.  Rows 0..8 are the elastic
// ones; rows 9 + 6l + i (memory variable i of mechanism l) use the stress-row
// Jacobian of the memory parameters (lambda, mu) -> (omega_l Ylam_l,
// omega_l Ymu_l).  On a face the memory rows take the elastic Godunov state:
// with d = q_R - q_L (face frame), its velocities are
//   v_n* = v_n,L + (d_nn + Zp_R d_vn) / (Zp_L + Zp_R),
//   v_s* = v_s,L + (d_ns + Zs_R d_vs) / (Zs_L + Zs_R)  (t alike),
// and the memory rows of the normal Jacobian only read velocities, so the
// memory flux is J_l (q_L + P d) with P's velocity rows above; rotated as
// stresses.
void visco_element(int64_t e, const double *X, const double *mats, const double *omega, const double *Ylam,
                   const double *Ymu, const int32_t *neigh, double *star, double *Ap, double *Am)
{
    const double *x = X + e * 12;
    double J[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) J[r][c] = x[(c + 1) * 3 + r] - x[r];
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
                     - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
                     + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    double G[3][3];
    G[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    G[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    G[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    G[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    G[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    G[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    G[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    G[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    G[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    const Mat mL = material(mats + e * 3);
    Mat mem[3];
    for (int l = 0; l < 3; ++l) {
        mem[l] = mL;
        mem[l].lam = omega[l] * Ylam[e * 3 + l];
        mem[l].mu = omega[l] * Ymu[e * 3 + l];
    }
    double *st = star + e * 3 * 27 * 9;
    std::memset(st, 0, sizeof(double) * 3 * 27 * 9);
    for (int d = 0; d < 3; ++d) {
        double A9[81] = {0};
        for (int j = 0; j < 3; ++j) add_jacobian(A9, j, mL, G[d][j]);
        for (int r = 0; r < 9; ++r)
            for (int c = 0; c < 9; ++c) st[(d * 27 + r) * 9 + c] = A9[r * 9 + c];
        for (int l = 0; l < 3; ++l) {
            double M9[81] = {0};
            for (int j = 0; j < 3; ++j) add_jacobian(M9, j, mem[l], G[d][j]);
            for (int r = 0; r < 6; ++r)
                for (int c = 0; c < 9; ++c) st[(d * 27 + 9 + 6 * l + r) * 9 + c] = M9[r * 9 + c];
        }
    }
    for (int s = 0; s < 4; ++s) {
        const double *a = x + FACEV[s][0] * 3, *b = x + FACEV[s][1] * 3, *c = x + FACEV[s][2] * 3;
        double ab[3], ac[3], cr[3];
        for (int k = 0; k < 3; ++k) { ab[k] = b[k] - a[k]; ac[k] = c[k] - a[k]; }
        cr[0] = ab[1] * ac[2] - ab[2] * ac[1];
        cr[1] = ab[2] * ac[0] - ab[0] * ac[2];
        cr[2] = ab[0] * ac[1] - ab[1] * ac[0];
        const double ncr = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        const double nab = std::sqrt(ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2]);
        double n[3], sv[3], t[3];
        for (int k = 0; k < 3; ++k) { n[k] = cr[k] / ncr; sv[k] = ab[k] / nab; }
        t[0] = n[1] * sv[2] - n[2] * sv[1];
        t[1] = n[2] * sv[0] - n[0] * sv[2];
        t[2] = n[0] * sv[1] - n[1] * sv[0];
        double Qm[3][3], Qt[3][3];
        for (int k = 0; k < 3; ++k) { Qm[k][0] = n[k]; Qm[k][1] = sv[k]; Qm[k][2] = t[k]; }
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) Qt[r][q] = Qm[q][r];
        double T[81], Ti[81];
        rotation(Qm, T);
        rotation(Qt, Ti);
        const int32_t nb = neigh[e * 4 + s];
        const Mat mR = material(mats + (nb >= 0 ? (int64_t)nb : e) * 3);
        const double ZpL = mL.rho * mL.cp, ZpR = mR.rho * mR.cp, ZsL = mL.rho * mL.cs, ZsR = mR.rho * mR.cs;
        const double iP = 1.0 / (ZpL + ZpR), iS = 1.0 / (ZsL + ZsR);
        // elastic rows (as dg_element_data_host)
        double W[81] = {0}, AL[81] = {0};
        add_jacobian(AL, 0, mL, 1.0);
        const double rP[9] = {mL.lam + 2 * mL.mu, mL.lam, mL.lam, 0, 0, 0, mL.cp, 0, 0};
        for (int r = 0; r < 9; ++r) {
            W[r * 9 + 0] -= rP[r] * iP;
            W[r * 9 + 6] -= rP[r] * ZpR * iP;
        }
        W[3 * 9 + 3] -= mL.mu * iS; W[3 * 9 + 7] -= mL.mu * ZsR * iS;
        W[7 * 9 + 3] -= mL.cs * iS; W[7 * 9 + 7] -= mL.cs * ZsR * iS;
        W[5 * 9 + 5] -= mL.mu * iS; W[5 * 9 + 8] -= mL.mu * ZsR * iS;
        W[8 * 9 + 5] -= mL.cs * iS; W[8 * 9 + 8] -= mL.cs * ZsR * iS;
        // velocity rows of the jump projector P (face frame)
        double Pv[3][9] = {{0}};
        Pv[0][0] = iP; Pv[0][6] = ZpR * iP;
        Pv[1][3] = iS; Pv[1][7] = ZsR * iS;
        Pv[2][5] = iS; Pv[2][8] = ZsR * iS;
        const double scale = -(ncr) / det;
        double *outp = Ap + (e * 4 + s) * 27 * 9, *outm = Am + (e * 4 + s) * 27 * 9;
        double Pp[81], tmp[81], res[81];
        for (int k = 0; k < 81; ++k) Pp[k] = AL[k] - W[k];
        matmul9(T, Pp, tmp);
        matmul9(tmp, Ti, res);
        for (int k = 0; k < 81; ++k) outp[(k / 9) * 9 + k % 9] = scale * res[k];
        matmul9(T, W, tmp);
        matmul9(tmp, Ti, res);
        for (int k = 0; k < 81; ++k) outm[(k / 9) * 9 + k % 9] = nb >= 0 ? scale * res[k] : 0.0;
        // memory rows: face frame F+ = Jl (I - P), F- = Jl P (only P's velocity
        // rows matter), then T_sigma F Ti
        for (int l = 0; l < 3; ++l) {
            double Jl[81] = {0};
            add_jacobian(Jl, 0, mem[l], 1.0);
            double Fp[81] = {0}, Fm[81] = {0};
            for (int r = 0; r < 6; ++r)
                for (int c = 0; c < 9; ++c) {
                    double pm = 0.0;
                    for (int v = 0; v < 3; ++v) pm += Jl[r * 9 + 6 + v] * Pv[v][c];
                    Fm[r * 9 + c] = pm;
                    Fp[r * 9 + c] = Jl[r * 9 + c] - pm;
                }
            for (int side = 0; side < 2; ++side) {
                const double *F = side ? Fm : Fp;
                double *out = side ? outm : outp;
                matmul9(T, F, tmp);          // rows 0..5: T_sigma F (F's rows 6..8 are zero)
                matmul9(tmp, Ti, res);
                for (int r = 0; r < 6; ++r)
                    for (int c = 0; c < 9; ++c)
                        out[(9 + 6 * l + r) * 9 + c] = (side && nb < 0) ? 0.0 : scale * res[r * 9 + c];
            }
        }
    }
}

}  // namespace

extern "C" int dg_visco_element_data_host(int64_t E, const double *X, const double *materials,
                                          const double *omega, const double *Ylam, const double *Ymu,
                                          const int32_t *neigh, double *star, double *Aplus, double *Aminus)
{
    if (E < 0 || (E > 0 && (!X || !materials || !omega || !Ylam || !Ymu || !neigh || !star || !Aplus || !Aminus)))
        return -1;
    unsigned nt = std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
    if (E < 4096) nt = 1;
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([=]() {
            for (int64_t e = t; e < E; e += nt) visco_element(e, X, materials, omega, Ylam, Ymu, neigh, star, Aplus, Aminus);
        });
    for (auto &x : th) x.join();
    return 0;
}

extern "C" int dg_element_data_host(int64_t E, const double *X, const double *materials,
                                    const int32_t *neigh, double *star, double *Aplus, double *Aminus)
{
    if (E < 0 || (E > 0 && (!X || !materials || !neigh || !star || !Aplus || !Aminus))) return -1;
    unsigned nt = std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
    if (E < 4096) nt = 1;
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([=]() {
            for (int64_t e = t; e < E; e += nt) one_element(e, X, materials, neigh, star, Aplus, Aminus);
        });
    for (auto &x : th) x.join();
    return 0;
}
