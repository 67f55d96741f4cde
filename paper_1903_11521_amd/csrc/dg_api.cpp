// C ABI of the element-kernel library: plans, argument checking, dispatch
// to the per-degree launch tables.  See include/dg.h for the contract.
#include "dg.h"

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <cstring>
#include <utility>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "dg_internal.h"
#include "refmat.h"
#include "visco_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, const char *what = nullptr, long long v = 0)
{
    char buf[512];
    std::snprintf(buf, sizeof buf, fmt, what ? what : "", v);
    g_err = buf;
    return code;
}

int hip_status(hipError_t e, const char *where)
{
    if (e == hipSuccess) return DG_OK;
    char buf[512];
    std::snprintf(buf, sizeof buf, "%s: HIP error %d (%s)", where, (int)e, hipGetErrorString(e));
    g_err = buf;
    return DG_EHIP;
}

// Synchronous validation of neighbour tables (off by default; see
// dg_set_debug_checks).  Copies the table to the host after the work already
// queued on the stream and checks every entry.
std::atomic<int> g_debug_checks{0};

int check_neighbours(const int32_t *neigh, int64_t E, int64_t bound, hipStream_t s, const char *who)
{
    if (!g_debug_checks.load() || E == 0) return DG_OK;
    std::vector<int32_t> h((size_t)E * 4);
    hipError_t e = hipMemcpyAsync(h.data(), neigh, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_status(e, who);
    for (int64_t i = 0; i < E * 4; ++i) {
        const int32_t v = h[(size_t)i];
        if (v < -1 || v >= bound) {
            char buf[256];
            std::snprintf(buf, sizeof buf, "%s: neighbour index %d of element %lld face %d outside [-1, %lld)", who,
                          (int)v, (long long)(i / 4), (int)(i % 4), (long long)bound);
            g_err = buf;
            return DG_EINVAL;
        }
    }
    return DG_OK;
}

#define CHECK_NEIGH(neigh, E, bound, s, who)                                        \
    do {                                                                            \
        const int rc_ = check_neighbours((neigh), (E), (bound), (s), (who));       \
        if (rc_ != DG_OK) return rc_;                                               \
    } while (0)

struct Tables {
    DgTable t[4][7];   // [precision][degree]
    Tables()
    {
        std::memset(t, 0, sizeof t);
        dg_table_2(&t[0][2], &t[1][2], &t[2][2]);
        dg_table_3(&t[0][3], &t[1][3], &t[2][3]);
        dg_table_4(&t[0][4], &t[1][4], &t[2][4]);
        dg_table_5(&t[0][5], &t[1][5], &t[2][5]);
        dg_table_6(&t[0][6], &t[1][6], &t[2][6]);
        dg_mtable_2(&t[3][2]);
        dg_mtable_3(&t[3][3]);
        dg_mtable_4(&t[3][4]);
        dg_mtable_5(&t[3][5]);
        dg_mtable_6(&t[3][6]);
        for (int n = 2; n <= 6; ++n) t[3][n].pack_star = t[1][n].pack_star;   // FP32 packed star
    }
};

const Tables &tables()
{
    static Tables t;
    return t;
}

bool aligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

DgItem make_item(int64_t E, double dt, void *Q, void *I, void *traces, const void *star, const double *Ap,
                 const double *Am, const int32_t *neigh, const uint8_t *fr)
{
    DgItem it;
    it.E = E;
    it.dt = dt;
    it.Q = Q;
    it.I = I;
    it.traces = traces;
    it.star = star;
    it.Ap = Ap;
    it.Am = Am;
    it.neigh = neigh;
    it.face_rot = fr;
    it.first_block = 0;
    it.nI = E;
    return it;
}

#define CHECK_PLAN(pl)                                                              \
    do {                                                                            \
        if (!(pl)) return fail(DG_EINVAL, "null plan%s", "");                       \
    } while (0)
#define CHECK_E(E)                                                                  \
    do {                                                                            \
        if ((E) < 0) return fail(DG_EINVAL, "negative element count%s %lld", "", (long long)(E)); \
        if ((E) > (int64_t)1 << 34) return fail(DG_EINVAL, "element count too large%s %lld", "", (long long)(E)); \
    } while (0)
#define CHECK_PTR(E, p, name)                                                       \
    do {                                                                            \
        if ((E) > 0 && !(p)) return fail(DG_EINVAL, "null pointer: %s", name);     \
        if ((E) > 0 && !aligned(p)) return fail(DG_EINVAL, "pointer not 16-byte aligned: %s", name); \
    } while (0)

}  // namespace

extern "C" {

const char *dg_last_error(void) { return g_err.c_str(); }

int64_t dg_reference_blob_size(int degree)
{
    if (degree < 1 || degree > 8) return -1;
    return (int64_t)dgref::blob_size(degree);
}

int dg_reference_matrices(int degree, double *out)
{
    if (degree < 1 || degree > 8) return fail(DG_EUNSUPPORTED, "degree %s%lld outside 1..8", "", degree);
    if (!out) return fail(DG_EINVAL, "null pointer: %s", "out");
    return dgref::build(degree, out) == 0 ? DG_OK : fail(DG_EINVAL, "reference matrix build failed%s", "");
}

int dg_plan_create(int degree, dg_precision precision, dg_plan **out)
{
    if (!out) return fail(DG_EINVAL, "null pointer: %s", "out");
    *out = nullptr;
    if (degree < 2 || degree > 6) return fail(DG_EUNSUPPORTED, "degree %s%lld outside 2..6", "", degree);
    if (precision != DG_FP64 && precision != DG_FP32 && precision != DG_MIXED && precision != DG_BF16X3)
        return fail(DG_EUNSUPPORTED, "unsupported precision %s%lld", "", (long long)precision);
    dg_plan *p = new (std::nothrow) dg_plan;
    if (!p) return fail(DG_ENOMEM, "out of host memory%s", "");
    p->degree = degree;
    p->prec = precision;
    p->B = dgref::basis_size(degree);
    p->Bf = dgref::face_basis_size(degree);
    p->tab = tables().t[precision][degree];
    *out = p;
    return DG_OK;
}

int dg_plan_destroy(dg_plan *plan)
{
    delete plan;
    return DG_OK;
}

int dg_plan_sizes(const dg_plan *plan, int *B, int *Bf)
{
    CHECK_PLAN(plan);
    if (B) *B = plan->B;
    if (Bf) *Bf = plan->Bf;
    return DG_OK;
}

int dg_pack_star(const dg_plan *plan, int64_t E, const double *star_dense, void *star_packed, hipStream_t s)
{
    CHECK_PLAN(plan);
    CHECK_E(E);
    CHECK_PTR(E, star_dense, "star_dense");
    CHECK_PTR(E, star_packed, "star_packed");
    return hip_status(plan->tab.pack_star(E, star_dense, star_packed, s), "dg_pack_star");
}

int dg_predictor(const dg_plan *plan, int64_t E, double dt, const void *Q, const void *star_packed, void *T,
                 hipStream_t s)
{
    CHECK_PLAN(plan);
    CHECK_E(E);
    CHECK_PTR(E, Q, "Q");
    CHECK_PTR(E, star_packed, "star_packed");
    CHECK_PTR(E, T, "T");
    if (!plan->tab.predictor) return fail(DG_EUNSUPPORTED, "dg_predictor: not available for this precision%s", "");
    return hip_status(plan->tab.predictor(E, dt, Q, star_packed, T, s), "dg_predictor");
}

int dg_time_integral(const dg_plan *plan, int64_t E, double dt, const void *T, void *I, hipStream_t s)
{
    CHECK_PLAN(plan);
    CHECK_E(E);
    CHECK_PTR(E, T, "T");
    CHECK_PTR(E, I, "I");
    if (!plan->tab.time_integral) return fail(DG_EUNSUPPORTED, "dg_time_integral: not available for this precision%s", "");
    return hip_status(plan->tab.time_integral(E, dt, T, I, s), "dg_time_integral");
}

int dg_volume(const dg_plan *plan, int64_t E, const void *I, const void *star_packed, void *Q, hipStream_t s)
{
    CHECK_PLAN(plan);
    CHECK_E(E);
    CHECK_PTR(E, I, "I");
    CHECK_PTR(E, star_packed, "star_packed");
    CHECK_PTR(E, Q, "Q");
    if (!plan->tab.volume) return fail(DG_EUNSUPPORTED, "dg_volume: not available for this precision%s", "");
    return hip_status(plan->tab.volume(E, I, star_packed, Q, s), "dg_volume");
}

int dg_local_flux(const dg_plan *plan, int64_t E, const void *I, const double *Aplus, void *Q, hipStream_t s)
{
    CHECK_PLAN(plan);
    CHECK_E(E);
    CHECK_PTR(E, I, "I");
    CHECK_PTR(E, Aplus, "Aplus");
    CHECK_PTR(E, Q, "Q");
    if (!plan->tab.local_flux) return fail(DG_EUNSUPPORTED, "dg_local_flux: not available for this precision%s", "");
    return hip_status(plan->tab.local_flux(E, I, Aplus, Q, s), "dg_local_flux");
}

int dg_neighbour_flux(const dg_plan *plan, int64_t E, int64_t n_I, const void *I, const int32_t *neigh,
                      const uint8_t *face_rot, const double *Aminus, void *Q, hipStream_t s)
{
    CHECK_PLAN(plan);
    CHECK_E(E);
    CHECK_E(n_I);
    if (E > 0 && n_I == 0) return fail(DG_EINVAL, "empty neighbour source array%s", "");
    CHECK_PTR(E, I, "I");
    CHECK_PTR(E, neigh, "neigh");
    CHECK_PTR(E, face_rot, "face_rot");
    CHECK_PTR(E, Aminus, "Aminus");
    CHECK_PTR(E, Q, "Q");
    CHECK_NEIGH(neigh, E, n_I, s, "dg_neighbour_flux");
    if (!plan->tab.neighbour_flux) return fail(DG_EUNSUPPORTED, "dg_neighbour_flux: not available for this precision%s", "");
    return hip_status(plan->tab.neighbour_flux(E, n_I, I, neigh, face_rot, Aminus, Q, s), "dg_neighbour_flux");
}

int dg_step(const dg_plan *plan, int64_t E, double dt, int n_steps, void *Q, void *I, void *traces,
            void *traces_b, const void *star_packed, const double *Aplus, const double *Aminus,
            const int32_t *neigh, const uint8_t *face_rot, hipStream_t s)
{
    return dg_step_impl(plan, E, dt, n_steps, Q, I, traces, traces_b, star_packed, Aplus, Aminus, neigh,
                        face_rot, s, true);
}

}  // extern "C"

int dg_set_error(int code, const char *msg)
{
    g_err = msg;
    return code;
}

int dg_step_impl(const dg_plan *plan, int64_t E, double dt, int n_steps, void *Q, void *I, void *traces,
                 void *traces_b, const void *star_packed, const double *Aplus, const double *Aminus,
                 const int32_t *neigh, const uint8_t *face_rot, hipStream_t s, bool debug_checks)
{
    CHECK_PLAN(plan);
    CHECK_E(E);
    if (n_steps < 0) return fail(DG_EINVAL, "negative step count%s %lld", "", n_steps);
    CHECK_PTR(E, Q, "Q");
    CHECK_PTR(E, I, "I");
    CHECK_PTR(E, traces, "traces");
    if (traces_b && (reinterpret_cast<uintptr_t>(traces_b) & 15))
        return fail(DG_EINVAL, "traces_b is not 16-byte aligned%s", "");
    if (traces_b && E > 0 && traces_b == traces) return fail(DG_EINVAL, "traces_b must not be traces%s", "");
    CHECK_PTR(E, star_packed, "star_packed");
    CHECK_PTR(E, Aplus, "Aplus");
    CHECK_PTR(E, Aminus, "Aminus");
    CHECK_PTR(E, neigh, "neigh");
    CHECK_PTR(E, face_rot, "face_rot");
    if (debug_checks) CHECK_NEIGH(neigh, E, E, s, "dg_step");
    if (!traces_b || n_steps < 2 || !plan->tab.fuse_step) {
        const DgItem it = make_item(E, dt, Q, I, traces, star_packed, Aplus, Aminus, neigh, face_rot);
        for (int n = 0; n < n_steps; ++n) {
            hipError_t e = plan->tab.step_predict(it, s);
            if (e != hipSuccess) return hip_status(e, "dg_step (predict)");
            e = plan->tab.step_correct(it, s);
            if (e != hipSuccess) return hip_status(e, "dg_step (correct)");
        }
        return DG_OK;
    }
    // predictor of step 1, then n-1 fused launches (corrector of step k and
    // predictor of step k+1), then the corrector of step n.  The traces
    // alternate between the two buffers; the first is chosen so that the
    // last step's traces end up in `traces`.
    void *cur = (n_steps & 1) ? traces : traces_b, *nxt = (n_steps & 1) ? traces_b : traces;
    DgItem it = make_item(E, dt, Q, I, cur, star_packed, Aplus, Aminus, neigh, face_rot);
    hipError_t e = plan->tab.step_predict(it, s);
    if (e != hipSuccess) return hip_status(e, "dg_step (predict)");
    for (int n = 1; n < n_steps; ++n) {
        e = plan->tab.step_fused(it, nxt, s);
        if (e != hipSuccess) return hip_status(e, "dg_step (fused)");
        std::swap(cur, nxt);
        it.traces = cur;
    }
    e = plan->tab.step_correct(it, s);
    if (e != hipSuccess) return hip_status(e, "dg_step (correct)");
    return DG_OK;
}

extern "C" {

int dg_step_predict(const dg_plan *plan, int64_t E, double dt, const void *Q, const void *star_packed, void *I,
                    void *traces, hipStream_t s)
{
    CHECK_PLAN(plan);
    CHECK_E(E);
    CHECK_PTR(E, Q, "Q");
    CHECK_PTR(E, star_packed, "star_packed");
    CHECK_PTR(E, I, "I");
    CHECK_PTR(E, traces, "traces");
    const DgItem it = make_item(E, dt, const_cast<void *>(Q), I, traces, star_packed, nullptr, nullptr, nullptr,
                                nullptr);
    return hip_status(plan->tab.step_predict(it, s), "dg_step_predict");
}

int dg_step_correct(const dg_plan *plan, int64_t E, const void *I, const void *traces, const void *star_packed,
                    const double *Aplus, const double *Aminus, const int32_t *neigh, const uint8_t *face_rot,
                    void *Q, hipStream_t s)
{
    CHECK_PLAN(plan);
    CHECK_E(E);
    CHECK_PTR(E, I, "I");
    CHECK_PTR(E, traces, "traces");
    CHECK_PTR(E, star_packed, "star_packed");
    CHECK_PTR(E, Aplus, "Aplus");
    CHECK_PTR(E, Aminus, "Aminus");
    CHECK_PTR(E, neigh, "neigh");
    CHECK_PTR(E, face_rot, "face_rot");
    CHECK_PTR(E, Q, "Q");
    CHECK_NEIGH(neigh, E, E, s, "dg_step_correct");
    const DgItem it = make_item(E, 0.0, Q, const_cast<void *>(I), const_cast<void *>(traces), star_packed, Aplus,
                                Aminus, neigh, face_rot);
    return hip_status(plan->tab.step_correct(it, s), "dg_step_correct");
}

int dg_step_fused(const dg_plan *plan, int64_t E, double dt, void *Q, void *I, const void *traces_in,
                  void *traces_out, const void *star_packed, const double *Aplus, const double *Aminus,
                  const int32_t *neigh, const uint8_t *face_rot, hipStream_t s)
{
    CHECK_PLAN(plan);
    CHECK_E(E);
    CHECK_PTR(E, Q, "Q");
    CHECK_PTR(E, I, "I");
    CHECK_PTR(E, traces_in, "traces_in");
    CHECK_PTR(E, traces_out, "traces_out");
    if (E > 0 && traces_in == traces_out) return fail(DG_EINVAL, "traces_out must not be traces_in%s", "");
    CHECK_PTR(E, star_packed, "star_packed");
    CHECK_PTR(E, Aplus, "Aplus");
    CHECK_PTR(E, Aminus, "Aminus");
    CHECK_PTR(E, neigh, "neigh");
    CHECK_PTR(E, face_rot, "face_rot");
    CHECK_NEIGH(neigh, E, E, s, "dg_step_fused");
    DgItem it = make_item(E, dt, Q, I, const_cast<void *>(traces_in), star_packed, Aplus, Aminus, neigh, face_rot);
    if (plan->tab.fuse_step) return hip_status(plan->tab.step_fused(it, traces_out, s), "dg_step_fused");
    // same work as two launches
    hipError_t e = plan->tab.step_correct(it, s);
    if (e != hipSuccess) return hip_status(e, "dg_step_fused (correct)");
    it.traces = traces_out;
    return hip_status(plan->tab.step_predict(it, s), "dg_step_fused (predict)");
}

int dg_fused_step(const dg_plan *plan, int64_t E, double dt, int n_steps, void *Q, void *I, void *traces,
                  const void *star_packed, const double *Aplus, const double *Aminus, const int32_t *neigh,
                  const uint8_t *face_rot, hipStream_t s)
{
    CHECK_PLAN(plan);
    if (!plan->tab.fused_predict || !plan->tab.fused_correct)
        return fail(DG_EUNSUPPORTED, "dg_fused_step: no fused-simulation form for this precision%s", "");
    CHECK_E(E);
    if (E > 0x7fffffff) return fail(DG_EINVAL, "dg_fused_step: element count too large%s %lld", "", (long long)E);
    if (n_steps < 0) return fail(DG_EINVAL, "negative step count%s %lld", "", n_steps);
    CHECK_PTR(E, Q, "Q");
    CHECK_PTR(E, I, "I");
    CHECK_PTR(E, traces, "traces");
    CHECK_PTR(E, star_packed, "star_packed");
    CHECK_PTR(E, Aplus, "Aplus");
    CHECK_PTR(E, Aminus, "Aminus");
    CHECK_PTR(E, neigh, "neigh");
    CHECK_PTR(E, face_rot, "face_rot");
    CHECK_NEIGH(neigh, E, E, s, "dg_fused_step");
    const DgItem it = make_item(E, dt, Q, I, traces, star_packed, Aplus, Aminus, neigh, face_rot);
    for (int n = 0; n < n_steps; ++n) {
        hipError_t e = plan->tab.fused_predict(it, s);
        if (e != hipSuccess) return hip_status(e, "dg_fused_step (predict)");
        e = plan->tab.fused_correct(it, s);
        if (e != hipSuccess) return hip_status(e, "dg_fused_step (correct)");
    }
    return DG_OK;
}

int dg_mra_apply(dg_precision precision, int64_t nb, int p, int q, const void *S, const void *XL, const void *XR,
                 const void *YL, const void *YR, const void *ZL, const void *ZR, void *R, hipStream_t s)
{
    if (precision != DG_FP64 && precision != DG_FP32)
        return fail(DG_EUNSUPPORTED, "dg_mra_apply: precision %s%lld is neither DG_FP64 nor DG_FP32", "",
                    (long long)precision);
    CHECK_E(nb);
    if (nb > 0x7fffffff) return fail(DG_EINVAL, "dg_mra_apply: batch too large%s %lld", "", (long long)nb);
    const int pmax = precision == DG_FP64 ? DG_MRA_MAX_P_FP64 : DG_MRA_MAX_P_FP32;
    if (p < 1 || p > pmax) return fail(DG_EUNSUPPORTED, "dg_mra_apply: tensor size p=%s%lld outside the supported range", "", p);
    if (q < 1 || q > p) return fail(DG_EINVAL, "dg_mra_apply: rank q=%s%lld outside 1..p", "", q);
    CHECK_PTR(nb, S, "S");
    CHECK_PTR(nb, R, "R");
    CHECK_PTR(nb, XL, "XL");
    CHECK_PTR(nb, XR, "XR");
    CHECK_PTR(nb, YL, "YL");
    CHECK_PTR(nb, YR, "YR");
    CHECK_PTR(nb, ZL, "ZL");
    CHECK_PTR(nb, ZR, "ZR");
    return hip_status(dg_mra_launch(precision == DG_FP64, nb, p, q, S, XL, XR, YL, YR, ZL, ZR, R, s), "dg_mra_apply");
}

int dg_plan_fuses_steps(const dg_plan *plan)
{
    CHECK_PLAN(plan);
    return plan->tab.fuse_step ? 1 : 0;
}

int dg_plan_set_fusion(dg_plan *plan, int fused)
{
    CHECK_PLAN(plan);
    if (fused != 0 && fused != 1) return fail(DG_EINVAL, "fusion mode %s%lld is neither 0 nor 1", "", fused);
    if (fused == 1 && !plan->tab.step_fused)
        return fail(DG_EUNSUPPORTED, "dg_plan_set_fusion: no fused step launch for this precision%s", "");
    plan->tab.fuse_step = fused == 1;
    return DG_OK;
}

int dg_set_debug_checks(int enable)
{
    return g_debug_checks.exchange(enable ? 1 : 0);
}

namespace {

// device work buffers of the tuner, freed on scope exit
struct TuneBuffers {
    std::vector<void *> p;
    ~TuneBuffers()
    {
        for (void *q : p) hipFree(q);
    }
    void *get(size_t bytes)
    {
        void *q = nullptr;
        if (hipMalloc(&q, bytes < 256 ? 256 : bytes) != hipSuccess) return nullptr;
        p.push_back(q);
        return q;
    }
};

}  // namespace

int dg_plan_tune(dg_plan *plan, int64_t E, hipStream_t s)
{
    CHECK_PLAN(plan);
    if (E < 64 || E > ((int64_t)1 << 26)) return fail(DG_EINVAL, "tuning size %s%lld outside [64, 2^26]", "", E);
    if (!plan->tab.step_fused) return 0;   // one schedule only (two launches)
    const size_t rs = plan->prec == DG_FP64 ? 8 : 4;
    const size_t nq = (size_t)E * 9 * plan->B, ntr = (size_t)E * 4 * 9 * plan->Bf;
    TuneBuffers b;
    void *Q = b.get(nq * rs), *I = b.get(nq * rs), *t0 = b.get(ntr * rs), *t1 = b.get(ntr * rs);
    void *star = b.get((size_t)E * 81 * rs);
    double *Ap = (double *)b.get((size_t)E * 4 * 81 * 8), *Am = (double *)b.get((size_t)E * 4 * 81 * 8);
    int32_t *neigh = (int32_t *)b.get((size_t)E * 4 * 4);
    uint8_t *rot = (uint8_t *)b.get((size_t)E * 4);
    if (!Q || !I || !t0 || !t1 || !star || !Ap || !Am || !neigh || !rot)
        return fail(DG_ENOMEM, "out of device memory%s for tuning", "");
    // zero data (kernel time does not depend on the values) on a neighbour
    // pattern with the reach of a structured mesh: faces point 1, 7, E/64 and
    // E/8 elements away
    std::vector<int32_t> nb((size_t)E * 4);
    const int64_t off[4] = {1, 7, E / 64 + 1, E / 8 + 1};
    for (int64_t e = 0; e < E; ++e)
        for (int f = 0; f < 4; ++f) nb[e * 4 + f] = (int32_t)((e + off[f]) % E);
    hipError_t e = hipMemcpyAsync(neigh, nb.data(), nb.size() * 4, hipMemcpyHostToDevice, s);
    for (void *z : {Q, I, t0, t1, star}) {
        if (e == hipSuccess) e = hipMemsetAsync(z, 0, z == star ? (size_t)E * 81 * rs : (z == Q || z == I) ? nq * rs : ntr * rs, s);
    }
    if (e == hipSuccess) e = hipMemsetAsync(Ap, 0, (size_t)E * 4 * 81 * 8, s);
    if (e == hipSuccess) e = hipMemsetAsync(Am, 0, (size_t)E * 4 * 81 * 8, s);
    if (e == hipSuccess) e = hipMemsetAsync(rot, 0, (size_t)E * 4, s);
    if (e != hipSuccess) return hip_status(e, "dg_plan_tune (setup)");
    const DgItem it = make_item(E, 1e-3, Q, I, t0, star, Ap, Am, neigh, rot);
    hipEvent_t ev[3];
    for (auto &x : ev)
        if ((e = hipEventCreate(&x)) != hipSuccess) return hip_status(e, "dg_plan_tune (events)");
    auto run = [&](bool fused) -> hipError_t {
        if (fused) return plan->tab.step_fused(it, t1, s);
        hipError_t r = plan->tab.step_correct(it, s);
        if (r == hipSuccess) {
            DgItem i2 = it;
            i2.traces = t1;
            r = plan->tab.step_predict(i2, s);
        }
        return r;
    };
    // warm both, then alternate 4 timed rounds of each; keep the faster total
    float tot[2] = {0.f, 0.f};
    for (int rep = -1; rep < 4 && e == hipSuccess; ++rep)
        for (int v = 0; v < 2 && e == hipSuccess; ++v) {
            e = hipEventRecord(ev[0], s);
            if (e == hipSuccess) e = run(v == 1);
            if (e == hipSuccess) e = hipEventRecord(ev[1], s);
            if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
            if (rep >= 0) tot[v] += ms;
        }
    for (auto &x : ev) hipEventDestroy(x);
    if (e != hipSuccess) return hip_status(e, "dg_plan_tune");
    plan->tab.fuse_step = tot[1] < tot[0];
    return plan->tab.fuse_step ? 1 : 0;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
}  // extern "C"

// A batch keeps two table slots.  Each holds, per degree present, the device
// item array and block-to-item table, and one step recorded into a HIP graph
// over them.  dg_batch_step replays the current slot; dg_batch_update writes
// the other slot (after the last replay that used it has finished), records
// its graph and makes it current, so the steps already enqueued keep reading
// the tables they were launched with and no device-wide wait is needed.
struct dg_batch {
    struct Group {
        int degree = 0;
        DgTable tab{};
        DgItem *d_items = nullptr;
        int32_t *d_block_item = nullptr;
        size_t cap_items = 0, cap_blocks = 0;
        int64_t n_items = 0, nblocks = 0;
    };
    struct VGroup {                // viscoelastic meshes of one degree
        VItem *d_items = nullptr;
        size_t cap = 0;
        int n_items = 0;
        int64_t total = 0;         // elements over the group's meshes
    };
    struct Slot {
        Group groups[7];           // by degree
        VGroup vgroups[7];
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipEvent_t last_use = nullptr;
        bool used = false;         // last_use recorded at least once
        bool empty = true;
    };
    dg_precision prec = DG_FP64;
    Slot slot[2];
    int cur = 0;
    hipStream_t aux = nullptr;     // private stream: table uploads and capture
    std::vector<DgItem> h_items;
    std::vector<int32_t> h_blocks;
    std::vector<VItem> h_vitems;
    double *vblob[7] = {};         // reference matrices of the viscoelastic degrees (device)
    ~dg_batch()
    {
        for (auto &sl : slot) {
            if (sl.last_use) (void)hipEventSynchronize(sl.last_use);
            if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
            if (sl.graph) (void)hipGraphDestroy(sl.graph);
            if (sl.last_use) (void)hipEventDestroy(sl.last_use);
            for (auto &g : sl.groups) {
                if (g.d_items) (void)hipFree(g.d_items);
                if (g.d_block_item) (void)hipFree(g.d_block_item);
            }
            for (auto &v : sl.vgroups)
                if (v.d_items) (void)hipFree(v.d_items);
        }
        for (double *p : vblob)
            if (p) (void)hipFree(p);
        if (aux) (void)hipStreamDestroy(aux);
    }
};

namespace {

bool is_visco(const dg_batch_item &x) { return x.n_quant == 27; }

int check_batch_items(dg_precision prec, const dg_batch_item *items, int n_items)
{
    if (n_items < 0 || (n_items > 0 && !items)) return fail(DG_EINVAL, "bad item list%s", "");
    for (int i = 0; i < n_items; ++i) {
        const dg_batch_item &x = items[i];
        if (x.degree < 2 || x.degree > 6) return fail(DG_EUNSUPPORTED, "item degree %s%lld outside 2..6", "", x.degree);
        if (x.n_quant != 0 && x.n_quant != 9 && x.n_quant != 27)
            return fail(DG_EINVAL, "item quantity count %s%lld is neither 9 nor 27", "", x.n_quant);
        if (is_visco(x)) {
            if (prec != DG_FP64)
                return fail(DG_EUNSUPPORTED, "viscoelastic items need a DG_FP64 batch%s", "");
            for (double w : x.omega)
                if (!(w >= 0.0) || w > 1e300)
                    return fail(DG_EINVAL, "item relaxation frequencies must be finite and >= 0%s", "");
        }
        CHECK_E(x.E);
        CHECK_PTR(x.E, x.Q, "item Q");
        CHECK_PTR(x.E, x.I, "item I");
        CHECK_PTR(x.E, x.traces, "item traces");
        CHECK_PTR(x.E, x.star_packed, "item star_packed");
        CHECK_PTR(x.E, x.Aplus, "item Aplus");
        CHECK_PTR(x.E, x.Aminus, "item Aminus");
        CHECK_PTR(x.E, x.neigh, "item neigh");
        CHECK_PTR(x.E, x.face_rot, "item face_rot");
        CHECK_NEIGH(x.neigh, x.E, x.E, nullptr, "dg_batch");
    }
    return DG_OK;
}

hipError_t ensure(void **p, size_t *cap, size_t bytes)
{
    if (*cap >= bytes && *p) return hipSuccess;
    size_t n = *cap ? *cap : 256;
    while (n < bytes) n *= 2;
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, n);
    if (e != hipSuccess) return e;
    if (*p) (void)hipFree(*p);   // only after the slot's last use has finished
    *p = q;
    *cap = n;
    return hipSuccess;
}

hipError_t batch_enqueue(const dg_batch *b, dg_batch::Slot &sl, hipStream_t s)
{
    for (auto &g : sl.groups) {
        if (!g.nblocks) continue;
        hipError_t e = g.tab.batch_predict(g.d_items, g.d_block_item, g.nblocks, s);
        if (e != hipSuccess) return e;
    }
    for (auto &g : sl.groups) {
        if (!g.nblocks) continue;
        hipError_t e = g.tab.batch_correct(g.d_items, g.d_block_item, g.nblocks, s);
        if (e != hipSuccess) return e;
    }
    for (int deg = 2; deg <= 6; ++deg) {
        const dg_batch::VGroup &v = sl.vgroups[deg];
        if (!v.total) continue;
        const VItem none{};
        hipError_t e = visco_step_launch(deg, v.d_items, v.n_items, none, v.total, b->vblob[deg], s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Writes `items` into slot k (whose last replay must have finished) and
// records its step graph.
int batch_fill(dg_batch *b, int k, const dg_batch_item *items, int n_items)
{
    dg_batch::Slot &sl = b->slot[k];
    if (sl.used) {
        hipError_t e = hipEventSynchronize(sl.last_use);
        if (e != hipSuccess) return hip_status(e, "dg_batch (slot wait)");
    }
    if (sl.exec) {
        (void)hipGraphExecDestroy(sl.exec);
        sl.exec = nullptr;
    }
    if (sl.graph) {
        (void)hipGraphDestroy(sl.graph);
        sl.graph = nullptr;
    }
    sl.empty = true;
    for (int deg = 2; deg <= 6; ++deg) {
        dg_batch::Group &G = sl.groups[deg];
        G.degree = deg;
        G.tab = tables().t[b->prec][deg];
        b->h_items.clear();
        b->h_blocks.clear();
        int64_t nb = 0;
        for (int i = 0; i < n_items; ++i) {
            const dg_batch_item &x = items[i];
            if (x.degree != deg || x.E == 0 || is_visco(x)) continue;
            DgItem it = make_item(x.E, x.dt, x.Q, x.I, x.traces, x.star_packed, x.Aplus, x.Aminus, x.neigh,
                                  x.face_rot);
            it.first_block = nb;
            const int64_t blocks = (x.E + DG_ELEMENTS_PER_BLOCK - 1) / DG_ELEMENTS_PER_BLOCK;
            for (int64_t q = 0; q < blocks; ++q) b->h_blocks.push_back((int32_t)b->h_items.size());
            nb += blocks;
            b->h_items.push_back(it);
        }
        if (nb > 0x7fffffff) return fail(DG_EINVAL, "batch too large%s", "");
        G.n_items = (int64_t)b->h_items.size();
        G.nblocks = nb;
        if (!nb) continue;
        sl.empty = false;
        hipError_t e = ensure(reinterpret_cast<void **>(&G.d_items), &G.cap_items, sizeof(DgItem) * b->h_items.size());
        if (e == hipSuccess)
            e = ensure(reinterpret_cast<void **>(&G.d_block_item), &G.cap_blocks, sizeof(int32_t) * b->h_blocks.size());
        if (e == hipSuccess)
            e = hipMemcpyAsync(G.d_items, b->h_items.data(), sizeof(DgItem) * b->h_items.size(),
                               hipMemcpyHostToDevice, b->aux);
        if (e == hipSuccess)
            e = hipMemcpyAsync(G.d_block_item, b->h_blocks.data(), sizeof(int32_t) * b->h_blocks.size(),
                               hipMemcpyHostToDevice, b->aux);
        // the host vectors are reused for the next degree: wait for this copy
        if (e == hipSuccess) e = hipStreamSynchronize(b->aux);
        if (e != hipSuccess) return hip_status(e, "dg_batch (tables)");
    }
    // viscoelastic meshes: one work list per degree
    for (int deg = 2; deg <= 6; ++deg) {
        dg_batch::VGroup &V = sl.vgroups[deg];
        b->h_vitems.clear();
        int64_t total = 0;
        for (int i = 0; i < n_items; ++i) {
            const dg_batch_item &x = items[i];
            if (x.degree != deg || x.E == 0 || !is_visco(x)) continue;
            VItem v{};
            v.E = x.E;
            v.first = total;
            v.dt = x.dt;
            for (int l = 0; l < 3; ++l) v.omega[l] = x.omega[l];
            v.Q = static_cast<double *>(x.Q), v.I = static_cast<double *>(x.I);
            v.traces = static_cast<double *>(x.traces);
            v.star = static_cast<const double *>(x.star_packed), v.Ap = x.Aplus, v.Am = x.Aminus;
            v.neigh = x.neigh, v.face_rot = x.face_rot;
            b->h_vitems.push_back(v);
            total += x.E;
        }
        V.n_items = (int)b->h_vitems.size();
        V.total = total;
        if (!total) continue;
        sl.empty = false;
        hipError_t e = hipSuccess;
        if (!b->vblob[deg]) {
            std::vector<double> blob(dgref::blob_size(deg));
            if (dgref::build(deg, blob.data()) != 0) return fail(DG_EINVAL, "reference matrix build failed%s", "");
            e = hipMalloc(reinterpret_cast<void **>(&b->vblob[deg]), blob.size() * sizeof(double));
            if (e == hipSuccess)
                e = hipMemcpyAsync(b->vblob[deg], blob.data(), blob.size() * sizeof(double), hipMemcpyHostToDevice,
                                   b->aux);
            if (e == hipSuccess) e = hipStreamSynchronize(b->aux);
        }
        if (e == hipSuccess)
            e = ensure(reinterpret_cast<void **>(&V.d_items), &V.cap, sizeof(VItem) * b->h_vitems.size());
        if (e == hipSuccess)
            e = hipMemcpyAsync(V.d_items, b->h_vitems.data(), sizeof(VItem) * b->h_vitems.size(),
                               hipMemcpyHostToDevice, b->aux);
        if (e == hipSuccess) e = hipStreamSynchronize(b->aux);
        if (e == hipSuccess) e = visco_prepare(deg);
        if (e != hipSuccess) return hip_status(e, "dg_batch (viscoelastic tables)");
    }
    if (sl.empty) return DG_OK;
    // record one step into a graph on the private stream
    hipError_t e = hipStreamBeginCapture(b->aux, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_status(e, "dg_batch (capture)");
    hipError_t le = batch_enqueue(b, sl, b->aux);
    e = hipStreamEndCapture(b->aux, &sl.graph);
    if (le != hipSuccess) return hip_status(le, "dg_batch (launch)");
    if (e == hipSuccess) e = hipGraphInstantiate(&sl.exec, sl.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_status(e, "dg_batch (instantiate)");
    return DG_OK;
}

}  // namespace

extern "C" {

int dg_batch_create(dg_precision precision, const dg_batch_item *items, int n_items, dg_batch **out)
{
    if (!out) return fail(DG_EINVAL, "null pointer: %s", "out");
    *out = nullptr;
    if (precision != DG_FP64 && precision != DG_FP32 && precision != DG_MIXED)
        return fail(DG_EUNSUPPORTED, "unsupported batch precision %s%lld", "", (long long)precision);
    int rc = check_batch_items(precision, items, n_items);
    if (rc != DG_OK) return rc;
    std::unique_ptr<dg_batch> b(new (std::nothrow) dg_batch);
    if (!b) return fail(DG_ENOMEM, "out of host memory%s", "");
    b->prec = precision;
    hipError_t e = hipStreamCreateWithFlags(&b->aux, hipStreamNonBlocking);
    for (auto &sl : b->slot)
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.last_use, hipEventDisableTiming);
    if (e != hipSuccess) return hip_status(e, "dg_batch_create");
    rc = batch_fill(b.get(), 0, items, n_items);
    if (rc != DG_OK) return rc;
    b->cur = 0;
    *out = b.release();
    return DG_OK;
}

int dg_batch_update(dg_batch *b, const dg_batch_item *items, int n_items)
{
    if (!b) return fail(DG_EINVAL, "null batch%s", "");
    int rc = check_batch_items(b->prec, items, n_items);
    if (rc != DG_OK) return rc;
    const int k = 1 - b->cur;
    rc = batch_fill(b, k, items, n_items);
    if (rc != DG_OK) return rc;
    b->cur = k;
    return DG_OK;
}

int dg_batch_step(dg_batch *b, int n_steps, hipStream_t s)
{
    if (!b) return fail(DG_EINVAL, "null batch%s", "");
    if (n_steps < 0) return fail(DG_EINVAL, "negative step count%s %lld", "", n_steps);
    dg_batch::Slot &sl = b->slot[b->cur];
    if (n_steps == 0 || sl.empty) return DG_OK;
    for (int n = 0; n < n_steps; ++n) {
        hipError_t e = hipGraphLaunch(sl.exec, s);
        if (e != hipSuccess) return hip_status(e, "dg_batch_step");
    }
    hipError_t e = hipEventRecord(sl.last_use, s);
    if (e != hipSuccess) return hip_status(e, "dg_batch_step (event)");
    sl.used = true;
    return DG_OK;
}

int dg_batch_destroy(dg_batch *b)
{
    delete b;
    return DG_OK;
}

int dg_sync(hipStream_t s) { return hip_status(hipStreamSynchronize(s), "dg_sync"); }

}  // extern "C"
