// C ABI of the viscoelastic step (27 quantities; see include/dg.h).
#include "dg.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>

#include "dg_internal.h"
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
