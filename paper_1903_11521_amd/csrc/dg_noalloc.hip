// dg_step_noalloc: dg_step with its face-trace work arrays in a fixed
// device buffer of the library, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops).  See
// include/dg.h for the contract.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "dg.h"
#include "dg_internal.h"

// The face-trace scratch of dg_step_noalloc.  Each device the library runs on
// holds its own copy until the process ends.  In host code this name is only
// a stand-in for the symbol: device code reaches the array through the
// per-device address taken below, never through the name.  (No `used`
// attribute: it would keep the symbol local to the code object, where the
// runtime's lookup by name cannot find it.)
static __device__ __align__(256) unsigned char scratch[DG_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];   // device address of `scratch` per device

// Address of the current device's copy of `scratch`, looked up once per
// device (with that device current) and kept.
int scratch_address(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "dg_step_noalloc: hipGetDevice failed: %s", hipGetErrorString(e));
        return dg_set_error(DG_EHIP, buf);
    }
    if (dev < 0 || dev >= kMaxDevices) return dg_set_error(DG_EUNSUPPORTED, "dg_step_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "dg_step_noalloc: hipGetSymbolAddress(scratch) failed: %s",
                          hipGetErrorString(e));
            return dg_set_error(DG_EHIP, buf);
        }
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return DG_OK;
}

}  // namespace

extern "C" int dg_step_noalloc(const dg_plan *plan, int64_t E, double dt, int n_steps, void *Q, void *I,
                               const void *star_packed, const double *Aplus, const double *Aminus,
                               const int32_t *neigh, const uint8_t *face_rot, hipStream_t stream)
{
    if (!plan) return dg_set_error(DG_EINVAL, "dg_step_noalloc: null plan");
    if (E < 0) return dg_set_error(DG_EINVAL, "dg_step_noalloc: negative element count");
    if (n_steps < 0) return dg_set_error(DG_EINVAL, "dg_step_noalloc: negative step count");
    const size_t rs = plan->prec == DG_FP64 ? 8 : 4;
    const unsigned long long one = (unsigned long long)E * 4ull * 9ull * (unsigned long long)plan->Bf * rs;
    if (one > (unsigned long long)DG_NOALLOC_SCRATCH_BYTES) {
        char buf[256];
        std::snprintf(buf, sizeof buf,
                      "dg_step_noalloc: %lld elements need %llu bytes of face traces, more than the fixed "
                      "scratch of %llu bytes (at most %lld elements for this plan)",
                      (long long)E, one, (unsigned long long)DG_NOALLOC_SCRATCH_BYTES,
                      (long long)(DG_NOALLOC_SCRATCH_BYTES / (4ull * 9ull * plan->Bf * rs)));
        return dg_set_error(DG_EINVAL, buf);
    }
    if (E == 0)
        return dg_step_impl(plan, E, dt, n_steps, Q, I, nullptr, nullptr, star_packed, Aplus, Aminus, neigh,
                            face_rot, stream, false);
    void *base = nullptr;
    const int rc = scratch_address(&base);
    if (rc != DG_OK) return rc;
    // the second trace array (one launch per step) only where the plan fuses
    // steps and both arrays fit; the two schedules give the same result
    const unsigned long long aligned = (one + 255ull) & ~255ull;
    void *tb = (plan->tab.fuse_step && 2ull * aligned <= (unsigned long long)DG_NOALLOC_SCRATCH_BYTES)
                   ? static_cast<void *>(static_cast<unsigned char *>(base) + aligned)
                   : nullptr;
    return dg_step_impl(plan, E, dt, n_steps, Q, I, base, tb, star_packed, Aplus, Aminus, neigh, face_rot, stream,
                        false);
}
