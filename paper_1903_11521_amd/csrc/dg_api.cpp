// C ABI of the element-kernel library: plans, argument checking, dispatch
// to the per-degree launch tables.  See include/dg.h for the contract.
#include "dg.h"

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "dg_internal.h"
#include "refmat.h"

struct dg_plan {
    int degree;
    dg_precision prec;
    int B, Bf;
    DgTable tab;
};

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

struct Tables {
    DgTable t64[7], t32[7];
    Tables()
    {
        std::memset(t64, 0, sizeof t64);
        std::memset(t32, 0, sizeof t32);
        dg_table_2(&t64[2], &t32[2]);
        dg_table_3(&t64[3], &t32[3]);
        dg_table_4(&t64[4], &t32[4]);
        dg_table_5(&t64[5], &t32[5]);
        dg_table_6(&t64[6], &t32[6]);
    }
};

const Tables &tables()
{
    static Tables t;
    return t;
}

bool aligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

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
    if (precision != DG_FP64 && precision != DG_FP32)
        return fail(DG_EUNSUPPORTED, "unsupported precision %s%lld", "", (long long)precision);
    dg_plan *p = new (std::nothrow) dg_plan;
    if (!p) return fail(DG_ENOMEM, "out of host memory%s", "");
    p->degree = degree;
    p->prec = precision;
    p->B = dgref::basis_size(degree);
    p->Bf = dgref::face_basis_size(degree);
    p->tab = precision == DG_FP64 ? tables().t64[degree] : tables().t32[degree];
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
    return hip_status(plan->tab.predictor(E, dt, Q, star_packed, T, s), "dg_predictor");
}

int dg_time_integral(const dg_plan *plan, int64_t E, double dt, const void *T, void *I, hipStream_t s)
{
    CHECK_PLAN(plan);
    CHECK_E(E);
    CHECK_PTR(E, T, "T");
    CHECK_PTR(E, I, "I");
    return hip_status(plan->tab.time_integral(E, dt, T, I, s), "dg_time_integral");
}

int dg_volume(const dg_plan *plan, int64_t E, const void *I, const void *star_packed, void *Q, hipStream_t s)
{
    CHECK_PLAN(plan);
    CHECK_E(E);
    CHECK_PTR(E, I, "I");
    CHECK_PTR(E, star_packed, "star_packed");
    CHECK_PTR(E, Q, "Q");
    return hip_status(plan->tab.volume(E, I, star_packed, Q, s), "dg_volume");
}

int dg_local_flux(const dg_plan *plan, int64_t E, const void *I, const double *Aplus, void *Q, hipStream_t s)
{
    CHECK_PLAN(plan);
    CHECK_E(E);
    CHECK_PTR(E, I, "I");
    CHECK_PTR(E, Aplus, "Aplus");
    CHECK_PTR(E, Q, "Q");
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
    return hip_status(plan->tab.neighbour_flux(E, n_I, I, neigh, face_rot, Aminus, Q, s), "dg_neighbour_flux");
}

int dg_step(const dg_plan *plan, int64_t E, double dt, int n_steps, void *Q, void *I, void *traces,
            const void *star_packed, const double *Aplus, const double *Aminus, const int32_t *neigh,
            const uint8_t *face_rot, hipStream_t s)
{
    CHECK_PLAN(plan);
    CHECK_E(E);
    if (n_steps < 0) return fail(DG_EINVAL, "negative step count%s %lld", "", n_steps);
    CHECK_PTR(E, Q, "Q");
    CHECK_PTR(E, I, "I");
    CHECK_PTR(E, traces, "traces");
    CHECK_PTR(E, star_packed, "star_packed");
    CHECK_PTR(E, Aplus, "Aplus");
    CHECK_PTR(E, Aminus, "Aminus");
    CHECK_PTR(E, neigh, "neigh");
    CHECK_PTR(E, face_rot, "face_rot");
    for (int n = 0; n < n_steps; ++n) {
        hipError_t e = plan->tab.step_predict(E, dt, Q, star_packed, I, traces, s);
        if (e != hipSuccess) return hip_status(e, "dg_step (predict)");
        e = plan->tab.step_correct(E, I, traces, star_packed, Aplus, Aminus, neigh, face_rot, Q, s);
        if (e != hipSuccess) return hip_status(e, "dg_step (correct)");
    }
    return DG_OK;
}

int dg_step_predict(const dg_plan *plan, int64_t E, double dt, const void *Q, const void *star_packed, void *I,
                    void *traces, hipStream_t s)
{
    CHECK_PLAN(plan);
    CHECK_E(E);
    CHECK_PTR(E, Q, "Q");
    CHECK_PTR(E, star_packed, "star_packed");
    CHECK_PTR(E, I, "I");
    CHECK_PTR(E, traces, "traces");
    return hip_status(plan->tab.step_predict(E, dt, Q, star_packed, I, traces, s), "dg_step_predict");
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
    return hip_status(plan->tab.step_correct(E, I, traces, star_packed, Aplus, Aminus, neigh, face_rot, Q, s),
                      "dg_step_correct");
}

int dg_sync(hipStream_t s) { return hip_status(hipStreamSynchronize(s), "dg_sync"); }

}  // extern "C"
