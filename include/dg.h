/*
 * dg.h - C ABI of the MI355X (gfx950) elastic ADER-DG element-kernel library.
 *
 * The library evaluates the element-local kernels of an ADER-DG scheme for
 * the linear elastic wave equation on unstructured tetrahedral meshes, as
 * written in Uphoff & Bader, "Yet Another Tensor Toolbox for discontinuous
 * Galerkin methods and other applications", Sec. 5.1.1:
 *   - the Cauchy-Kowalevski predictor        (Eq. seissol:derivative)
 *   - the Taylor time integral               (Eq. seissol:timeint)
 *   - the volume and local flux terms        (Eq. seissol:correction_local)
 *   - the neighbour flux term                (Eq. seissol:correction_neigh)
 *
 * Conventions
 *   degree N in 2..6;  B = (N+1)(N+2)(N+3)/6 volume and Bf = (N+1)(N+2)/2
 *   face basis functions (Sec. 5.1.1); 9 quantities in the order
 *   s_xx s_yy s_zz s_xy s_yz s_xz u v w (velocity-stress form of Eq.
 *   linearpde).  Basis: Dubiner's functions on the reference tetrahedron
 *   (0,0,0),(1,0,0),(0,1,0),(0,0,1) in the collapsed-coordinate Jacobi form,
 *   ordered by total degree, then by the zeta index, then by the eta index.
 *   Local face s of an element is the local-vertex triple (0,2,1), (0,1,3),
 *   (0,3,2), (1,2,3) with outward normal (x_b-x_a)x(x_c-x_a).
 *
 *   All DOF-like arrays are element major, basis index fastest:
 *     Q, I      [E][9][B]          DOFs, time integral
 *     T         [E][N+1][9][B]     Taylor-scaled time derivatives
 *                                  T^d = dt^d/d! * D^d  (rows of T^d at or
 *                                  beyond C(N-d+3,3) are written as 0)
 *     traces    [E][4][9*Bf]       face traces R^s^T I of every element; one
 *                                  face block holds the face basis in parts
 *                                  of whole degree blocks, one part after the
 *                                  other, each part quantity major
 *                                  ([9][rows of the part]).  FP32, mixed and
 *                                  BF16X3 plans use one part ([9][Bf]); FP64 plans
 *                                  split the face basis into parts of at most
 *                                  16 rows (degree 5: rows [0,15), [15,21);
 *                                  degree 6: [0,15), [15,28)).
 *     star_packed [E][9][3][3]     star matrices in packed form (see
 *                                  dg_pack_star), element type of the plan
 *     Aplus, Aminus [E][4][9][9]   flux-solver matrices, FP64, row major
 *                                  (row = output quantity), geometric factor
 *                                  -2|S|/det J and rotation folded in
 *     neigh     [E][4] int32       neighbour element of each face (-1: none;
 *                                  then that face's neighbour term is 0)
 *     face_rot  [E][4] uint8       j | h << 2: the neighbour's local face j
 *                                  and the orientation h (position of this
 *                                  face's first vertex in the neighbour's
 *                                  face triple)
 *   The element type of DOF arrays is double for DG_FP64 plans and float for
 *   DG_FP32, DG_MIXED and DG_BF16X3 plans.
 *
 * Memory and streams: every array argument of the dg_* compute calls is a
 * DEVICE pointer owned by the caller; the library does not allocate, free or
 * retain caller memory.  Calls are enqueued on the caller's hipStream_t and
 * return before the GPU work completes.  Host-side helpers (suffix _host and
 * dg_reference_matrices) take host pointers and run synchronously.
 *
 * Errors: every call returns a dg_status.  Argument errors (null pointer,
 * negative size, unsupported degree or precision, misaligned pointer) are
 * reported synchronously and nothing is enqueued.  A failed kernel launch
 * returns DG_EHIP; faults during execution surface from dg_sync.  The text
 * of the last error of the calling thread is available from dg_last_error.
 * Plans are immutable after creation (except for dg_plan_tune and
 * dg_plan_set_fusion) and may be shared between threads.
 */
#ifndef DG_H
#define DG_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_plan dg_plan;

/* DG_FP64: everything in FP64.  DG_FP32: DOFs, star matrices and every
 * contraction in FP32 (flux solvers are read as FP64 and rounded).
 * DG_MIXED: FP32 DOFs and reference-matrix contractions; the Taylor time
 * integral is accumulated in FP64 and the flux-solver products run in FP64
 * (rounded once to FP32).
 * DG_BF16X3: FP32 DOFs and star matrices; every reference-matrix contraction
 * runs on the matrix cores as three BF16 products, A_hi B_hi + A_hi B_lo +
 * A_lo B_hi (x_hi = bf16(x), x_lo = bf16(x - x_hi), round to nearest even),
 * accumulated in FP32, about 3 * 2^-16 relative error per product; the
 * flux-solver products run in FP64 (rounded once to FP32); the Taylor scale
 * factors dt/(k+1) and the dt*Q term of the time integral are formed in FP64
 * and rounded once, the derivative terms added in FP32.  Only the step
 * launches (dg_step, dg_step_predict, dg_step_correct, dg_step_noalloc, with
 * two launches per step) and dg_pack_star exist for it; the per-stage calls,
 * dg_step_fused's one-launch form and batches return DG_EUNSUPPORTED.
 * DOF-like arrays are float for FP32, MIXED and BF16X3. */
typedef enum { DG_FP64 = 0, DG_FP32 = 1, DG_MIXED = 2, DG_BF16X3 = 3 } dg_precision;

typedef enum {
    DG_OK = 0,
    DG_EINVAL = -1,
    DG_EUNSUPPORTED = -2,
    DG_EHIP = -3,
    DG_ENOMEM = -4
} dg_status;

/* ---- host helpers ------------------------------------------------------ */

/* Number of doubles written by dg_reference_matrices for `degree`. */
int64_t dg_reference_blob_size(int degree);

/* Reference matrices of Sec. 5.1.1 for `degree` (host, FP64, row major),
 * concatenated: Khat[3][B][B], Ktilde[3][B][B], R[4][B][Bf], Rhat[4][B][Bf],
 * f[3][Bf][Bf], mass[B], face_mass[Bf].  Khat^d = M^-1 S^d and
 * Ktilde^d = -M^-1 S^d^T with S^d_kl = int dphi_k/dxi_d phi_l; R^s_ln is the
 * face-basis projection of phi_l on face s, Rhat^s = M^-1 R^s Mf, f^h maps
 * face coefficients between the two orientations of a shared face.
 * `out` must hold dg_reference_blob_size(degree) doubles. */
int dg_reference_matrices(int degree, double *out);

/* Star matrices and flux solvers of every element (host, FP64).
 * X [E][4][3] vertex coordinates, materials [E][3] = (rho, cp, cs),
 * neigh [E][4].  Writes star [E][3][9][9] (A*^d = sum_j dxi_d/dx_j A^(j),
 * Sec. 5.1.1), Aplus and Aminus [E][4][9][9] (exact Godunov flux between the
 * element's and the neighbour's isotropic materials).  Host pointers. */
/* Viscoelastic element data (three mechanisms; 27 quantities: the 9
 * elastic ones, then 6 memory variables per mechanism).  omega [3] the
 * mechanisms' relaxation frequencies, Ylam, Ymu [E][3] their coefficients;
 * star [E][3][27][9] and Aplus, Aminus [E][4][27][9]: the rows of all 27
 * quantities over the 9 elastic columns (the only ones the operators read).
 * Memory rows: the stress rows of the Jacobians with (lambda, mu) replaced by
 * (omega_l Ylam_l, omega_l Ymu_l); on faces they take the elastic Godunov
 * state.  Host arrays; returns 0, or -1 for a null pointer or E < 0. */
int dg_visco_element_data_host(int64_t E, const double *X, const double *materials, const double *omega,
                               const double *Ylam, const double *Ymu, const int32_t *neigh, double *star,
                               double *Aplus, double *Aminus);
int dg_element_data_host(int64_t E, const double *X, const double *materials, const int32_t *neigh,
                         double *star, double *Aplus, double *Aminus);

/* ---- plans ------------------------------------------------------------- */

int dg_plan_create(int degree, dg_precision precision, dg_plan **out);
int dg_plan_destroy(dg_plan *plan);
/* B and Bf of a plan (either pointer may be NULL). */
int dg_plan_sizes(const dg_plan *plan, int *B, int *Bf);
/* 1 if this plan runs dg_step_fused (and dg_step with a second trace array)
 * as one fused launch, 0 if as two launches (the faster choice, measured on
 * MI355X: fused from degree 2 to 3); negative status on a null plan. */
int dg_plan_fuses_steps(const dg_plan *plan);
/* Launch-schedule tuner: times dg_step_fused as one fused launch and as two
 * launches (corrector, then predictor) on E synthetic elements of this
 * plan's degree and precision, and keeps the faster for this plan.  Returns
 * 1 (fused) or 0 (two launches), or a negative status.  Allocates and frees
 * its own device work buffers (about E times the per-element footprint) and
 * synchronises the stream.  Call it before the plan is shared between
 * threads (it and dg_plan_set_fusion are the only calls that change a
 * plan).  E in [64, 2^26]. */
int dg_plan_tune(dg_plan *plan, int64_t E, hipStream_t stream);
/* Sets the launch schedule of dg_step (with a second trace array) and
 * dg_step_fused: fused = 1 runs step k's corrector and step k+1's predictor as
 * one launch, fused = 0 as two launches.  Both give the same result bit for
 * bit; the choice only changes speed.  Like dg_plan_tune it changes the plan:
 * call it before the plan is shared between threads.  DG_EINVAL if fused is
 * neither 0 nor 1. */
int dg_plan_set_fusion(dg_plan *plan, int fused);
const char *dg_last_error(void);

/* Debug checks (process wide, off by default; returns the previous setting).
 * When on, every call that takes a neighbour table (dg_neighbour_flux,
 * dg_step, dg_step_correct, dg_step_fused, dg_batch_create) first waits for
 * the work already queued on its stream, copies the table to the host and
 * returns DG_EINVAL, with the offending element and face in dg_last_error and
 * nothing enqueued, if an entry lies outside [-1, bound) (bound = n_I for
 * dg_neighbour_flux, E otherwise).  With the checks off such entries are
 * treated like -1 (no neighbour) and are not reported. */
int dg_set_debug_checks(int enable);

/* ---- device compute calls (stream ordered) ----------------------------- */

/* Packs dense FP64 star matrices [E][3][9][9] into the plan's packed form
 * [E][9][3][3]: entry [p][d][i] is star^d[p][q_i(p)] with the elastic
 * coupling columns q(p) = (6,7,8) for p<3, (6,7,-) p=3, (7,8,-) p=4,
 * (6,8,-) p=5, (0,3,5) p=6, (1,3,4) p=7, (2,4,5) p=8 ('-' stored as 0).
 * Entries of the dense matrices outside this pattern are ignored. */
int dg_pack_star(const dg_plan *plan, int64_t E, const double *star_dense, void *star_packed,
                 hipStream_t stream);

/* Eq. seissol:derivative: T[e][d] = dt^d/d! D^d for d = 0..N, D^0 = Q. */
int dg_predictor(const dg_plan *plan, int64_t E, double dt, const void *Q, const void *star_packed,
                 void *T, hipStream_t stream);

/* Eq. seissol:timeint: I = sum_d dt/(d+1) T^d, accumulated in FP64.  T is
 * the Taylor-scaled derivative array of dg_predictor; rows of T^d at and past
 * C(N-d+3, 3) (the staircase, zero for every derivative of the predictor)
 * are not read. */
int dg_time_integral(const dg_plan *plan, int64_t E, double dt, const void *T, void *I,
                     hipStream_t stream);

/* Eq. seissol:correction_local, stiffness part: Q += sum_d Khat^d I star^d^T. */
int dg_volume(const dg_plan *plan, int64_t E, const void *I, const void *star_packed, void *Q,
              hipStream_t stream);

/* Eq. seissol:correction_local, face part: Q += sum_s Rhat^s (R^s^T I) Aplus^s^T. */
int dg_local_flux(const dg_plan *plan, int64_t E, const void *I, const double *Aplus, void *Q,
                  hipStream_t stream);

/* Eq. seissol:correction_neigh:
 * Q += sum_s Rhat^s f^h (R^j^T I[neigh]) Aminus^s^T, (j,h) from face_rot.
 * I [n_I][9][B] holds the time integrals of the elements neigh refers to;
 * neighbour indices outside [0, n_I) are treated like -1 (no neighbour). */
int dg_neighbour_flux(const dg_plan *plan, int64_t E, int64_t n_I, const void *I, const int32_t *neigh,
                      const uint8_t *face_rot, const double *Aminus, void *Q, hipStream_t stream);

/* n_steps global time steps of the full scheme (predictor, time integral,
 * volume, local and neighbour flux) on all E elements, Q updated in place.
 * I [E][9][B] and traces [E][4][9*Bf] are caller-provided work arrays; on
 * return they hold the time integral and face traces of the last step.
 * traces_b (same size as traces, or NULL) is a second trace array.  With it,
 * and where dg_plan_fuses_steps says so, step k's corrector and step k+1's
 * predictor run as one launch (one launch per step; the traces alternate
 * between the two arrays, because neighbours still read step k's traces
 * while step k+1's are written).  Otherwise each step is two launches.  All
 * give the same result bit for bit.  Neighbour indices must lie in [0, E)
 * or be -1; others are treated like -1, or rejected with DG_EINVAL when the
 * debug checks are on (dg_set_debug_checks). */
int dg_step(const dg_plan *plan, int64_t E, double dt, int n_steps, void *Q, void *I, void *traces,
            void *traces_b, const void *star_packed, const double *Aplus, const double *Aminus,
            const int32_t *neigh, const uint8_t *face_rot, hipStream_t stream);

/* The two launches of one dg_step, exposed separately so that a caller can
 * place work (for instance an exchange of partition-boundary traces) between
 * them.  dg_step_predict: I = time integral of the predictor of Q and
 * traces[e][s] = R^s^T I[e] (face block layout above; a face block is
 * contiguous, so it can be exchanged as one piece).  dg_step_correct: Q +=
 * volume + local flux +
 * neighbour flux, the local and neighbour terms read from `traces`. */
int dg_step_predict(const dg_plan *plan, int64_t E, double dt, const void *Q, const void *star_packed,
                    void *I, void *traces, hipStream_t stream);
int dg_step_correct(const dg_plan *plan, int64_t E, const void *I, const void *traces,
                    const void *star_packed, const double *Aplus, const double *Aminus,
                    const int32_t *neigh, const uint8_t *face_rot, void *Q, hipStream_t stream);

/* The launch between them in a fused dg_step: the corrector of step k
 * (reading I and the step-k traces in traces_in; Q += volume + local flux +
 * neighbour flux) followed, per element in the same launch, by the predictor
 * of step k+1 on the updated Q (I overwritten with step k+1's time integral,
 * its traces written to traces_out, which must not be traces_in: neighbours
 * still read traces_in).  dg_step_predict, then n-1 dg_step_fused with the
 * trace arrays swapped after each, then dg_step_correct, is n steps.  Where
 * dg_plan_fuses_steps is 0 the two halves run as two launches. */
int dg_step_fused(const dg_plan *plan, int64_t E, double dt, void *Q, void *I, const void *traces_in,
                  void *traces_out, const void *star_packed, const double *Aplus, const double *Aminus,
                  const int32_t *neigh, const uint8_t *face_rot, hipStream_t stream);

/* ---- fused simulations -------------------------------------------------- */

/* Number of simulations a fused step advances together. */
#define DG_FUSED_SIMS 16

/* n_steps time steps of DG_FUSED_SIMS independent simulations on one mesh:
 * the extra simulation index s of the paper's multiple-simulation form
 * (Sec. 3 and 5.1.1: every DOF tensor Q_kp gains an index s, Q_kps, and the
 * element-local operators act on all s alike).  The simulations share the
 * mesh, the star matrices and the flux solvers; they differ in their DOFs.
 * Only for DG_BF16X3 plans (DG_EUNSUPPORTED otherwise): the reference
 * matrices meet the 16 simulations of one element on the matrix cores, so a
 * wave reads each element's star matrices, flux solvers and neighbour
 * relation once for all 16.  Layouts (float, simulation index fastest):
 *     Q, I    [E][9][B][16]
 *     traces  [E][4][9][Bf][16]   (work array)
 * and star_packed, Aplus, Aminus, neigh, face_rot as for dg_step.  Each
 * simulation's result is bit for bit that of dg_step with the same plan on
 * that simulation's DOFs.  E < 2^31. */
int dg_fused_step(const dg_plan *plan, int64_t E, double dt, int n_steps, void *Q, void *I, void *traces,
                  const void *star_packed, const double *Aplus, const double *Aminus, const int32_t *neigh,
                  const uint8_t *face_rot, hipStream_t stream);

/* ---- the separable contraction of Sec. 7 -------------------------------- */

/* Largest tensor size p of dg_mra_apply (two p^3 tensors held in LDS). */
#define DG_MRA_MAX_P_FP64 20
#define DG_MRA_MAX_P_FP32 24

/* Eq. stock_mra (the MADNESS kernel of Sec. 7) for a batch of nb tensors:
 *     R_ijk = sum S_xyz X^L_xl X^R_li Y^L_ym Y^R_mj Z^L_zn Z^R_nk
 * with i, j, k, x, y, z in 0..p-1 and l, m, n in 0..q-1 (1 <= q <= p), the six
 * operator factors shared by the batch.  Device pointers, row major, element
 * type double (DG_FP64) or float (DG_FP32):  S, R [nb][p][p][p];
 * XL, YL, ZL [p][q];  XR, YR, ZR [q][p].  Evaluated as the paper's chain of
 * six one-index contractions on the matrix cores, FP64 or FP32 throughout
 * (products and sums), one workgroup per tensor.  p up to DG_MRA_MAX_P_FP64
 * or DG_MRA_MAX_P_FP32 (DG_EUNSUPPORTED above). */
int dg_mra_apply(dg_precision precision, int64_t nb, int p, int q, const void *S, const void *XL, const void *XR,
                 const void *YL, const void *YR, const void *ZL, const void *ZR, void *R, hipStream_t stream);

/* ---- local time stepping ------------------------------------------------ */

/* Clustered local time stepping of rate 2 (Sec. 6.4, Table tab:loh1 compares
 * it with global time stepping).  Element e belongs to cluster cluster[e]
 * and steps with dt0 * 2^cluster[e]; face neighbours must differ by at most
 * one cluster, and elements must be numbered cluster by cluster
 * (non-decreasing cluster ids).  Each step of an element is the ADER step of
 * Eqs. seissol:derivative, seissol:timeint, seissol:correction_local and
 * seissol:correction_neigh, except that the neighbour term integrates each
 * neighbour's predicted solution over the element's own step: the
 * neighbour's step integral (same cluster), the half of its Taylor expansion
 * that the step covers (larger cluster), or the sum of its two step
 * integrals (smaller cluster).  One cycle is 2^(C-1) steps of the smallest
 * cluster, C the number of clusters (max cluster id + 1); after each cycle
 * all elements are at the same time. */
#define DG_LTS_MAX_CLUSTERS 16
typedef struct dg_lts dg_lts;

/* Builds the schedule: cluster ranges and, per cluster, the neighbours whose
 * integrals it gathers.  cluster [E] and neigh [E][4] (indices in [-1, E))
 * are HOST arrays, read during the call only.  Allocates the work arrays
 * (Taylor-scaled derivatives [E][N+1][9][B] and three [E][9][B] arrays of
 * the plan's storage type) in device memory owned by the handle.  Errors:
 * DG_EUNSUPPORTED for a precision without per-stage kernels (DG_BF16X3),
 * DG_EINVAL for unsorted clusters, ids outside [0, DG_LTS_MAX_CLUSTERS),
 * neighbours two or more clusters apart or a non-positive dt0, DG_ENOMEM. */
int dg_lts_create(const dg_plan *plan, int64_t E, const int32_t *cluster, const int32_t *neigh, double dt0,
                  dg_lts **out);
/* Number of clusters and element updates per cycle (sum over clusters of
 * their size times 2^(C-1-c)); either output may be NULL. */
int dg_lts_clusters(const dg_lts *lts, int *n_clusters, int64_t *updates_per_cycle);
/* Advances Q [E][9][B] (device, updated in place) by n_cycles cycles on
 * `stream`.  The static arrays are those of dg_step for the same E elements
 * (device pointers, 16-byte aligned).  The handle's work arrays make
 * concurrent calls on one handle race. */
int dg_lts_advance(dg_lts *lts, int n_cycles, void *Q, const void *star_packed, const double *Aplus,
                   const double *Aminus, const int32_t *neigh, const uint8_t *face_rot, hipStream_t stream);
/* Frees the handle and its device memory (after the caller's stream work
 * that uses it has finished). */
int dg_lts_destroy(dg_lts *lts);

/* ---- viscoelastic elements ------------------------------------------------ */

/* n_steps global steps of the viscoelastic scheme (27 quantities: the 9
 * elastic ones, then 3 mechanisms x 6 memory variables; Sec. 5.1 names the
 * rheology): the ADER step of Eqs. seissol:derivative, seissol:timeint,
 * seissol:correction_local and seissol:correction_neigh with 27 rows, plus
 * the source terms D^d E^T in the derivative recursion and I E^T in the
 * update (E: stress rows -sum_l theta_l, memory rows -omega_l theta_l), and
 * no derivative staircase.  FP64 device arrays: Q, I [E][27][B] (Q updated
 * in place, I work), traces [E][4][9][Bf] work (the elastic face traces of
 * I), star [E][3][27][9], Aplus, Aminus [E][4][27][9] (from
 * dg_visco_element_data_host), ref the blob of dg_reference_matrices for
 * the degree copied to the device, neigh [E][4] (indices outside [0, E): no
 * neighbour), face_rot [E][4] = j | h << 2 (orientations above 2 are invalid
 * and read as 0); omega [3] a HOST array of the relaxation frequencies.
 * Degrees 2..6.  Persistent workgroups walk the elements in the launch shape
 * of the degree (dg_visco_tune, dg_visco_set_shape).  Errors, before
 * anything is enqueued: DG_EUNSUPPORTED for the degree; DG_EINVAL for E
 * outside [0, 2^31), a negative step count, a null pointer, a negative or
 * non-finite omega or a non-finite dt; DG_EHIP if a launch fails. */
int dg_visco_step(int degree, int64_t E, double dt, int n_steps, double *Q, double *I, double *traces,
                  const double *star, const double *Aplus, const double *Aminus, const double *omega,
                  const double *ref, const int32_t *neigh, const uint8_t *face_rot, hipStream_t stream);

/* ---- LinA: ADER-DG-SEM on cuboids ---------------------------------------- */

/* The LinA scheme (Sec. 5.2): linear acoustics (quantities p, u, v, w) on a
 * uniform periodic grid of cubes of edge h, tensor-product nodal basis on
 * the `order` Gauss-Lobatto points per direction (degree order-1).  One time
 * step is Eq. lina:derivative and Eq. lina:integration (the predictor and its
 * time integral I), the weak derivatives Q* = Q + Kh I A* + ..., the side
 * values of Eq. lin3d_evaluateSide and the side fluxes of Eq. lina3d_flux. */
#define DG_LINA_MAX_ORDER_FP64 12
#define DG_LINA_MAX_ORDER_FP32 16

/* Number of doubles of a coefficient blob of the given order (-1 if outside
 * [2, DG_LINA_MAX_ORDER_FP32]). */
int64_t dg_lina_blob_size(int order);
/* Fills the host FP64 coefficient blob: Kt [O][O] (minus the collocation
 * derivative), Kh [O][O] (the weak derivative M^-1 S), the Gauss-Lobatto
 * weights w [O] on [0, 1], the star matrices [3][4][4] (A/h, B/h, C/h of
 * density rho0 and bulk modulus K0) and the upwind side flux solvers
 * Ap, Am [6][4][4] (sides left, right, bottom, top, back, front; geometric
 * factor -1/h folded in). */
int dg_lina_coefficients(int order, double rho0, double K0, double h, double *out);
/* n_steps time steps of dt.  Q [E][4][order][order][order] (x fastest),
 * updated in place; sides [E][6][4][order][order] a work array (on return:
 * the side values of the last step's time integral); coef the blob above
 * copied to the device in the step's precision (double for DG_FP64, float
 * for DG_FP32); neigh [E][6] the neighbour across each side (indices in
 * [0, E); others drop that side's neighbour term).  Only the acoustic pattern of the
 * star matrices is read (entries (0, 1+d) and (1+d, 0) of direction d).
 * Orders up to DG_LINA_MAX_ORDER_FP64 / _FP32; device pointers, stream
 * ordered. */
int dg_lina_step(dg_precision precision, int order, int64_t E, int n_steps, double dt, void *Q, void *sides,
                 const double *coef, const int32_t *neigh, hipStream_t stream);

/* Launch-shape tuner of the viscoelastic kernels (the batched form's tiles
 * and elements per workgroup).  Both kernels keep one element per workgroup
 * in flight and walk the work list with persistent workgroups; the shape is
 * the number of waves per workgroup (4 or 8: how an element's 16x16 tiles are
 * spread) and the number of resident workgroups per CU (elements in flight
 * per CU, up to what LDS and registers admit).  Times every candidate for
 * `degree` on E synthetic elements (allocates and frees device memory, and
 * synchronizes `stream`) and keeps the fastest for the process: later
 * dg_visco_step calls, and batches created or updated afterwards, use it.
 * The shape never changes an element's arithmetic (results are bitwise the
 * same).  waves / groups_per_cu (may be null) receive the choice.
 * E in [64, 2^22] (the device memory it needs grows with E and the degree:
 * about 66 KB per element at degree 6; DG_ENOMEM if it does not fit).  The
 * shape table is process-wide and not synchronised: tune or set shapes
 * before other threads launch viscoelastic steps. */
int dg_visco_tune(int degree, int64_t E, hipStream_t stream, int *waves, int *groups_per_cu);
/* Sets the launch shape of a degree without timing (for example one saved
 * from an earlier dg_visco_tune): waves 4 or 8, groups_per_cu 0 (as many as
 * fit) or a cap in [1, 64] (capped again at what fits).  Host only; later
 * steps and batches created or updated afterwards use it. */
int dg_visco_set_shape(int degree, int waves, int groups_per_cu);
/* The current launch shape of a degree (waves, groups_per_cu may be null). */
int dg_visco_get_shape(int degree, int *waves, int *groups_per_cu);

/* ---- batches of independent meshes (mixed degrees) --------------------- */

/* One mesh of a batch.  All pointers are device pointers owned by the caller
 * and must stay valid for the batch's lifetime.  Elastic items (n_quant 9):
 * layouts as for dg_step with the item's degree, element type per the batch
 * precision.  Viscoelastic items (n_quant 27, DG_FP64 batches only): layouts
 * as for dg_visco_step, FP64: Q and I [E][27][B], traces [E][4][9][Bf],
 * star_packed the viscoelastic star matrices [E][3][27][9] and Aplus, Aminus
 * [E][4][27][9] as dg_visco_element_data_host writes them, and omega the
 * relaxation frequencies of the item's three mechanisms. */
typedef struct {
    int degree;                 /* 2..6 */
    int64_t E;                  /* elements of this mesh (>= 0) */
    double dt;                  /* time step of this mesh */
    void *Q, *I, *traces;       /* DOFs (updated in place) and work arrays */
    const void *star_packed;
    const double *Aplus, *Aminus;
    const int32_t *neigh;       /* indices local to this mesh, in [0, E) */
    const uint8_t *face_rot;
    int n_quant;                /* 9 (elastic; 0 is read as 9) or 27 (viscoelastic) */
    double omega[3];            /* viscoelastic items: relaxation frequencies (finite, >= 0) */
} dg_batch_item;

typedef struct dg_batch dg_batch;

/* Builds the work tables of a batch (device memory owned by the batch; this
 * call allocates, and uploads on a private stream that it waits for).  One
 * time step of a batch is one predictor launch and one corrector launch per
 * degree and material model present, over all meshes of that degree and
 * model (the viscoelastic launches are persistent workgroups walking the
 * elements of all their meshes); the launches of a step are recorded once
 * into a HIP graph and replayed.  Each element's arithmetic is identical to
 * dg_step's (elastic) or dg_visco_step's (viscoelastic), so a mesh gives
 * bitwise the same result alone and in any batch.  DG_EUNSUPPORTED for a
 * viscoelastic item in a batch that is not DG_FP64. */
int dg_batch_create(dg_precision precision, const dg_batch_item *items, int n_items, dg_batch **out);
/* n_steps time steps of every mesh of the batch, stream ordered. */
int dg_batch_step(dg_batch *batch, int n_steps, hipStream_t stream);
/* Replaces the batch's mesh list (continuous batching: meshes join and
 * leave between steps).  Steps enqueued after this call step the new list;
 * steps enqueued before it still read the old one.  The batch keeps two
 * copies of its work tables and step graph and writes the one not used by
 * the latest dg_batch_step, after the replays that used it have finished
 * (a host wait on that slot only, not on the device); the tables are
 * uploaded on a private stream and the step graph is recorded again.  No
 * device-wide synchronisation.  Meshes that stay in the batch give bitwise
 * the same results as before the update. */
int dg_batch_update(dg_batch *batch, const dg_batch_item *items, int n_items);
int dg_batch_destroy(dg_batch *batch);

/* ---- stepping without device allocation ------------------------------ */

/* Size in bytes of the library's fixed per-device face-trace buffer used by
 * dg_step_noalloc (256 MiB). */
#define DG_NOALLOC_SCRATCH_BYTES (256ull << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): dg_step
 * without the caller's face-trace work arrays.  The traces live in a
 * library-owned device buffer of DG_NOALLOC_SCRATCH_BYTES, one copy per
 * device, held from the library's load until the process ends; its address
 * on the current device is looked up on the first call on that device.  The
 * call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine) and skips the dg_set_debug_checks neighbour validation, which
 * would copy the table to host memory.  Q, I and the static data are as for
 * dg_step (I holds the last step's time integral on return); the result is
 * bit for bit that of dg_step.  E times one trace array (E*4*9*Bf values of
 * the plan's element type) must fit the buffer, else DG_EINVAL with the
 * limit in dg_last_error and nothing enqueued (degree 5: 44 385 elements in
 * FP64, 88 770 in FP32, mixed or BF16X3).  With two trace arrays' room, and where the
 * plan fuses steps, one launch per step; otherwise two.  The buffer keeps the
 * previous call's traces; every step writes all traces before any is read,
 * so nothing needs clearing.  All calls on one device share the buffer:
 * calls that overlap on a device (different streams, or threads without
 * ordering) race and give wrong results. */
int dg_step_noalloc(const dg_plan *plan, int64_t E, double dt, int n_steps, void *Q, void *I,
                    const void *star_packed, const double *Aplus, const double *Aminus,
                    const int32_t *neigh, const uint8_t *face_rot, hipStream_t stream);

/* Waits for the stream; reports asynchronous kernel failures as DG_EHIP. */
int dg_sync(hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* DG_H */
