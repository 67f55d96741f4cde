// C ABI of the viscoelastic step (27 quantities; see include/dg.h).
#include "dg.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "dg_internal.h"
#include "refmat.h"
#include "visco_internal.h"

extern "C" int dg_visco_step(int degree, int64_t E, double dt, int n_steps, double *Q, double *I, double *traces,
                             const double *star, const double *Aplus, const double *Aminus, const double *omega,
                             const double *ref, const int32_t *neigh, const uint8_t *face_rot, hipStream_t stream)
{
    char buf[256];
    if (degree < 2 || degree > 6) {
        std::snprintf(buf, sizeof buf, "dg_visco_step: degree %d outside 2..6", degree);
        return dg_set_error(DG_EUNSUPPORTED, buf);
    }
    if (E < 0 || E > 0x7fffffff || n_steps < 0)
        return dg_set_error(DG_EINVAL, "dg_visco_step: element or step count out of range");
    if (E == 0 || n_steps == 0) return DG_OK;
    if (!Q || !I || !traces || !star || !Aplus || !Aminus || !omega || !ref || !neigh || !face_rot)
        return dg_set_error(DG_EINVAL, "dg_visco_step: null pointer");
    VItem one{};
    one.E = E;
    one.first = 0;
    one.dt = dt;
    for (int l = 0; l < 3; ++l) {
        if (!std::isfinite(omega[l]) || omega[l] < 0.0)
            return dg_set_error(DG_EINVAL, "dg_visco_step: relaxation frequencies must be finite and >= 0");
        one.omega[l] = omega[l];
    }
    if (!std::isfinite(dt)) return dg_set_error(DG_EINVAL, "dg_visco_step: dt not finite");
    one.Q = Q, one.I = I, one.traces = traces;
    one.star = star, one.Ap = Aplus, one.Am = Aminus;
    one.neigh = neigh, one.face_rot = face_rot;
    for (int s = 0; s < n_steps; ++s) {
        const hipError_t e = visco_step_launch(degree, nullptr, 1, one, E, ref, stream);
        if (e != hipSuccess) {
            std::snprintf(buf, sizeof buf, "dg_visco_step: HIP error %d (%s)", (int)e, hipGetErrorString(e));
            return dg_set_error(DG_EHIP, buf);
        }
    }
    return DG_OK;
}

namespace {

// device buffers of the tuning run, freed on every return path
struct TuneMem {
    std::vector<void *> p;
    void *get(size_t bytes)
    {
        void *q = nullptr;
        if (hipMalloc(&q, bytes) != hipSuccess) return nullptr;
        p.push_back(q);
        return q;
    }
    ~TuneMem()
    {
        for (void *q : p) (void)hipFree(q);
    }
};

int tune_fail(hipError_t e)
{
    char buf[256];
    std::snprintf(buf, sizeof buf, "dg_visco_tune: HIP error %d (%s)", (int)e, hipGetErrorString(e));
    return dg_set_error(DG_EHIP, buf);
}

}  // namespace

extern "C" int dg_visco_tune(int degree, int64_t E, hipStream_t stream, int *waves, int *groups_per_cu)
{
    char buf[256];
    if (degree < 2 || degree > 6) {
        std::snprintf(buf, sizeof buf, "dg_visco_tune: degree %d outside 2..6", degree);
        return dg_set_error(DG_EUNSUPPORTED, buf);
    }
    if (E < 64 || E > ((int64_t)1 << 22)) return dg_set_error(DG_EINVAL, "dg_visco_tune: tuning size outside [64, 2^22]");
    const int64_t B = dgref::basis_size(degree), Bf = dgref::face_basis_size(degree);
    TuneMem m;
    double *Q = (double *)m.get((size_t)E * 27 * B * 8), *I = (double *)m.get((size_t)E * 27 * B * 8);
    double *tr = (double *)m.get((size_t)E * 36 * Bf * 8), *star = (double *)m.get((size_t)E * 3 * 27 * 9 * 8);
    double *Ap = (double *)m.get((size_t)E * 4 * 27 * 9 * 8), *Am = (double *)m.get((size_t)E * 4 * 27 * 9 * 8);
    int32_t *neigh = (int32_t *)m.get((size_t)E * 16);
    uint8_t *rot = (uint8_t *)m.get((size_t)E * 4);
    const size_t nblob = dgref::blob_size(degree);
    double *blob = (double *)m.get(nblob * 8);
    if (!Q || !I || !tr || !star || !Ap || !Am || !neigh || !rot || !blob)
        return dg_set_error(DG_ENOMEM, "dg_visco_tune: out of device memory");
    // zero data (the kernels' time does not depend on the values), the
    // product's reference matrices, and neighbours 1, 7, E/64 and E/8 away
    std::vector<double> hb(nblob);
    if (dgref::build(degree, hb.data()) != 0) return dg_set_error(DG_EINVAL, "dg_visco_tune: reference matrices");
    std::vector<int32_t> nb((size_t)E * 4);
    const int64_t off[4] = {1, 7, E / 64 + 1, E / 8 + 1};
    for (int64_t e = 0; e < E; ++e)
        for (int f = 0; f < 4; ++f) nb[(size_t)(e * 4 + f)] = (int32_t)((e + off[f]) % E);
    hipError_t e = hipMemcpyAsync(blob, hb.data(), nblob * 8, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(neigh, nb.data(), nb.size() * 4, hipMemcpyHostToDevice, stream);
    for (auto z : {std::make_pair((void *)Q, (size_t)E * 27 * B * 8), std::make_pair((void *)I, (size_t)E * 27 * B * 8),
                   std::make_pair((void *)tr, (size_t)E * 36 * Bf * 8),
                   std::make_pair((void *)star, (size_t)E * 3 * 27 * 9 * 8),
                   std::make_pair((void *)Ap, (size_t)E * 4 * 27 * 9 * 8),
                   std::make_pair((void *)Am, (size_t)E * 4 * 27 * 9 * 8), std::make_pair((void *)rot, (size_t)E * 4)})
        if (e == hipSuccess) e = hipMemsetAsync(z.first, 0, z.second, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return tune_fail(e);
    VItem one{};
    one.E = E, one.first = 0, one.dt = 1e-3;
    one.Q = Q, one.I = I, one.traces = tr, one.star = star, one.Ap = Ap, one.Am = Am, one.neigh = neigh;
    one.face_rot = rot;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    VShape best{0, 0};
    float best_ms = 0.0f;
    for (int w : {4, 8}) {
        int maxpc = 0;
        if (e == hipSuccess) e = visco_prepare_shape(degree, w, &maxpc);
        for (int pc = 1; e == hipSuccess && pc <= maxpc; ++pc) {
            const VShape sh{w, pc};
            e = visco_step_shape(degree, sh, nullptr, 1, one, E, blob, stream);    // warm-up
            if (e == hipSuccess) e = hipEventRecord(t0, stream);
            for (int r = 0; r < 3 && e == hipSuccess; ++r) e = visco_step_shape(degree, sh, nullptr, 1, one, E, blob, stream);
            if (e == hipSuccess) e = hipEventRecord(t1, stream);
            if (e == hipSuccess) e = hipEventSynchronize(t1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
            if (e == hipSuccess && (best.waves == 0 || ms < best_ms)) best = sh, best_ms = ms;
        }
    }
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (e != hipSuccess) return tune_fail(e);
    visco_set_shape(degree, best);
    if (waves) *waves = best.waves;
    if (groups_per_cu) *groups_per_cu = best.per_cu;
    return DG_OK;
}

extern "C" int dg_visco_set_shape(int degree, int waves, int groups_per_cu)
{
    if (degree < 2 || degree > 6) return dg_set_error(DG_EUNSUPPORTED, "dg_visco_set_shape: degree outside 2..6");
    if (waves != 4 && waves != 8) return dg_set_error(DG_EINVAL, "dg_visco_set_shape: waves must be 4 or 8");
    if (groups_per_cu < 0 || groups_per_cu > 64)
        return dg_set_error(DG_EINVAL, "dg_visco_set_shape: workgroups per CU outside [0, 64]");
    visco_set_shape(degree, VShape{waves, groups_per_cu});
    return DG_OK;
}

extern "C" int dg_visco_get_shape(int degree, int *waves, int *groups_per_cu)
{
    if (degree < 2 || degree > 6) return dg_set_error(DG_EUNSUPPORTED, "dg_visco_get_shape: degree outside 2..6");
    const VShape sh = visco_shape(degree);
    if (waves) *waves = sh.waves;
    if (groups_per_cu) *groups_per_cu = sh.per_cu;
    return DG_OK;
}
