/*
 * Oracle stage loop nests (TEST INFRASTRUCTURE: only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark load this library).
 *
 * Plain FP64 evaluation of the element-local ADER-DG stages of the paper's
 * Sec. 5.1.1, over FULL index ranges (no zero-block skipping, no fusion),
 * OpenMP only over elements.  Every multi-factor Einstein term is evaluated as
 * the fixed sequence of binary contractions written next to it.
 *
 * Array layouts (row-major C arrays):
 *   reference: Kt, Kh [3][B][B]; R, Rh [4][B][Bf]; f [3][Bf][Bf]
 *   per element: star [E][3][P][P]; Ap, Am [E][4][P][P]
 *   DOFs: Q, I, dQ [E][P][B]  (basis index fastest);  D [E][N+1][P][B]
 *   neighbours: neigh [E][4] (int32, -1 = none), nface, orient [E][4] (int8)
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX3(a, b, c, nb, nc) (((size_t)(a) * (nb) + (b)) * (nc) + (c))

/* Number of OpenMP threads of the loops below (timing runs only). */
void oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int oracle_max_threads(void) { return omp_get_max_threads(); }

/* Eq. seissol:derivative:  D^{d+1}_kp = sum_xi Kt^xi_kl D^d_lq Astar^xi_pq,
 * evaluated as  tmp_lp = D_lq Astar_pq  then  D'_kp += Kt_kl tmp_lp.      */
void oracle_predictor(int N, int B, int P, int64_t E, const double *Kt,
                      const double *star, const double *Q, double *D)
{
#pragma omp parallel
    {
        double *tmp = (double *)malloc(sizeof(double) * B * P);
#pragma omp for schedule(static)
        for (int64_t e = 0; e < E; ++e) {
            double *De = D + (size_t)e * (N + 1) * P * B;
            memcpy(De, Q + (size_t)e * P * B, sizeof(double) * P * B);
            for (int d = 0; d < N; ++d) {
                const double *Dc = De + (size_t)d * P * B;
                double *Dn = De + (size_t)(d + 1) * P * B;
                memset(Dn, 0, sizeof(double) * P * B);
                for (int xi = 0; xi < 3; ++xi) {
                    const double *A = star + IDX3(e, xi, 0, 3, P * P);
                    const double *K = Kt + (size_t)xi * B * B;
                    for (int l = 0; l < B; ++l)
                        for (int p = 0; p < P; ++p) {
                            double s = 0.0;
                            for (int q = 0; q < P; ++q) s += Dc[q * B + l] * A[p * P + q];
                            tmp[l * P + p] = s;
                        }
                    for (int k = 0; k < B; ++k)
                        for (int p = 0; p < P; ++p) {
                            double s = 0.0;
                            for (int l = 0; l < B; ++l) s += K[k * B + l] * tmp[l * P + p];
                            Dn[p * B + k] += s;
                        }
                }
            }
        }
        free(tmp);
    }
}

/* Eq. seissol:timeint:  I = sum_{d=0}^{N} dt^{d+1}/(d+1)! D^d. */
void oracle_time_integral(int N, int B, int P, int64_t E, double dt,
                          const double *D, double *I)
{
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        const double *De = D + (size_t)e * (N + 1) * P * B;
        double *Ie = I + (size_t)e * P * B;
        for (int i = 0; i < P * B; ++i) {
            double coef = 1.0, s = 0.0;
            for (int d = 0; d <= N; ++d) {
                coef *= dt / (double)(d + 1);
                s += coef * De[(size_t)d * P * B + i];
            }
            Ie[i] = s;
        }
    }
}

/* Eq. seissol:correction_local, volume part:
 * dQ_kp = sum_xi Kh^xi_kl I_lq Astar^xi_pq  as  tmp_lp = I_lq Astar_pq;
 * dQ_kp += Kh_kl tmp_lp.  dQ is overwritten. */
void oracle_volume(int B, int P, int64_t E, const double *Kh, const double *star,
                   const double *I, double *dQ)
{
#pragma omp parallel
    {
        double *tmp = (double *)malloc(sizeof(double) * B * P);
#pragma omp for schedule(static)
        for (int64_t e = 0; e < E; ++e) {
            const double *Ie = I + (size_t)e * P * B;
            double *out = dQ + (size_t)e * P * B;
            memset(out, 0, sizeof(double) * P * B);
            for (int xi = 0; xi < 3; ++xi) {
                const double *A = star + IDX3(e, xi, 0, 3, P * P);
                const double *K = Kh + (size_t)xi * B * B;
                for (int l = 0; l < B; ++l)
                    for (int p = 0; p < P; ++p) {
                        double s = 0.0;
                        for (int q = 0; q < P; ++q) s += Ie[q * B + l] * A[p * P + q];
                        tmp[l * P + p] = s;
                    }
                for (int k = 0; k < B; ++k)
                    for (int p = 0; p < P; ++p) {
                        double s = 0.0;
                        for (int l = 0; l < B; ++l) s += K[k * B + l] * tmp[l * P + p];
                        out[p * B + k] += s;
                    }
            }
        }
        free(tmp);
    }
}

/* one face term  dQ_kp += Rh_km [ (F_mn (R_ln I_lq)) Aflux_pq ]  with F = I
 * when f == NULL.  t1_nq = R_ln I_lq ; t2_mq = F_mn t1_nq ; t3_mp = t2_mq A_pq ;
 * dQ_kp += Rh_km t3_mp. */
static void face_term(int B, int Bf, int P, const double *Rh, const double *R,
                      const double *f, const double *Iin, const double *A,
                      double *t1, double *t2, double *t3, double *out)
{
    for (int n = 0; n < Bf; ++n)
        for (int q = 0; q < P; ++q) {
            double s = 0.0;
            for (int l = 0; l < B; ++l) s += R[l * Bf + n] * Iin[q * B + l];
            t1[n * P + q] = s;
        }
    const double *t = t1;
    if (f) {
        for (int m = 0; m < Bf; ++m)
            for (int q = 0; q < P; ++q) {
                double s = 0.0;
                for (int n = 0; n < Bf; ++n) s += f[m * Bf + n] * t1[n * P + q];
                t2[m * P + q] = s;
            }
        t = t2;
    }
    for (int m = 0; m < Bf; ++m)
        for (int p = 0; p < P; ++p) {
            double s = 0.0;
            for (int q = 0; q < P; ++q) s += t[m * P + q] * A[p * P + q];
            t3[m * P + p] = s;
        }
    for (int k = 0; k < B; ++k)
        for (int p = 0; p < P; ++p) {
            double s = 0.0;
            for (int m = 0; m < Bf; ++m) s += Rh[k * Bf + m] * t3[m * P + p];
            out[p * B + k] += s;
        }
}

/* Eq. seissol:correction_local, flux part (R-tilde read as R). dQ overwritten. */
void oracle_local_flux(int B, int Bf, int P, int64_t E, const double *Rh,
                       const double *R, const double *Ap, const double *I, double *dQ)
{
#pragma omp parallel
    {
        double *t1 = (double *)malloc(sizeof(double) * Bf * P * 3);
        double *t2 = t1 + Bf * P, *t3 = t2 + Bf * P;
#pragma omp for schedule(static)
        for (int64_t e = 0; e < E; ++e) {
            double *out = dQ + (size_t)e * P * B;
            memset(out, 0, sizeof(double) * P * B);
            for (int s = 0; s < 4; ++s)
                face_term(B, Bf, P, Rh + (size_t)s * B * Bf, R + (size_t)s * B * Bf, NULL,
                          I + (size_t)e * P * B, Ap + IDX3(e, s, 0, 4, P * P), t1, t2, t3, out);
        }
        free(t1);
    }
}

/* Eq. seissol:correction_neigh:  (nu, j, h) = (neigh, nface, orient)[e][s].
 * Faces with neigh < 0 contribute nothing.  dQ overwritten. */
void oracle_neighbour_flux(int B, int Bf, int P, int64_t E, const double *Rh,
                           const double *R, const double *f, const int32_t *neigh,
                           const int8_t *nface, const int8_t *orient,
                           const double *Am, const double *I, double *dQ)
{
#pragma omp parallel
    {
        double *t1 = (double *)malloc(sizeof(double) * Bf * P * 3);
        double *t2 = t1 + Bf * P, *t3 = t2 + Bf * P;
#pragma omp for schedule(static)
        for (int64_t e = 0; e < E; ++e) {
            double *out = dQ + (size_t)e * P * B;
            memset(out, 0, sizeof(double) * P * B);
            for (int s = 0; s < 4; ++s) {
                int32_t nu = neigh[e * 4 + s];
                if (nu < 0) continue;
                int j = nface[e * 4 + s], h = orient[e * 4 + s];
                face_term(B, Bf, P, Rh + (size_t)s * B * Bf, R + (size_t)j * B * Bf,
                          f + (size_t)h * Bf * Bf, I + (size_t)nu * P * B,
                          Am + IDX3(e, s, 0, 4, P * P), t1, t2, t3, out);
            }
        }
        free(t1);
    }
}
