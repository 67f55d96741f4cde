// Launchers of the split-BF16 matrix-core step kernels for one polynomial
// degree (DG_DEGREE).  Compiled once per supported degree.
#include <cstring>

#include "dg_tables.h"
#include "mfma_kernels.hip"

#ifndef DG_DEGREE
#error "DG_DEGREE must be defined"
#endif

namespace {

constexpr int N = DG_DEGREE;

unsigned tile_blocks(int64_t E) { return (unsigned)((E + dgm::EPT - 1) / dgm::EPT); }

hipError_t step_predict(const DgItem &it, hipStream_t s)
{
    if (it.E == 0) return hipSuccess;
    hipLaunchKernelGGL((dgm::k_mstep_predict<N, false>), dim3(tile_blocks(it.E)), dim3(64), 0, s, it.E, it.dt,
                       (const float *)it.Q, (const float *)it.star, (float *)it.I, (float *)it.traces);
    return hipGetLastError();
}

hipError_t step_correct(const DgItem &it, hipStream_t s)
{
    if (it.E == 0) return hipSuccess;
    hipLaunchKernelGGL((dgm::k_mstep_correct<N, false>), dim3(tile_blocks(it.E)), dim3(64), 0, s, it.E,
                       (const float *)it.I, (const float *)it.traces, (const float *)it.star, it.Ap, it.Am,
                       it.neigh, it.face_rot, (float *)it.Q);
    return hipGetLastError();
}

// fused simulations: one element (16 simulations) per wave
hipError_t fused_predict(const DgItem &it, hipStream_t s)
{
    if (it.E == 0) return hipSuccess;
    hipLaunchKernelGGL((dgm::k_mstep_predict<N, true>), dim3((unsigned)it.E), dim3(64), 0, s, it.E, it.dt,
                       (const float *)it.Q, (const float *)it.star, (float *)it.I, (float *)it.traces);
    return hipGetLastError();
}

hipError_t fused_correct(const DgItem &it, hipStream_t s)
{
    if (it.E == 0) return hipSuccess;
    hipLaunchKernelGGL((dgm::k_mstep_correct<N, true>), dim3((unsigned)it.E), dim3(64), 0, s, it.E,
                       (const float *)it.I, (const float *)it.traces, (const float *)it.star, it.Ap, it.Am,
                       it.neigh, it.face_rot, (float *)it.Q);
    return hipGetLastError();
}

}  // namespace

#define DG_CAT2(a, b) a##b
#define DG_CAT(a, b) DG_CAT2(a, b)

// DG_BF16X3 table: the two step launches and their fused-simulation form
// (star packing is the FP32 plans', filled in by the caller)
void DG_CAT(dg_mtable_, DG_DEGREE)(DgTable *t)
{
    std::memset(t, 0, sizeof *t);
    t->step_predict = step_predict;
    t->step_correct = step_correct;
    t->fused_predict = fused_predict;
    t->fused_correct = fused_correct;
    t->fuse_step = false;
}
