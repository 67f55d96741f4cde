// Launchers of the local-time-stepping kernels (lts_kernels.hip), used by
// the scheduler in lts.cpp.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Weights of the Taylor-scaled derivatives for an integral over part of a
// step (at most degree 6, so at most 7 derivatives).
struct LtsWeights {
    double w[8];
};

hipError_t dg_lts_gather(bool fp64, int64_t n, int PB, int N1, const int32_t *ids, const int8_t *kind,
                         const void *T, const void *I, const void *Buf, void *G, const LtsWeights &w, hipStream_t s);
hipError_t dg_lts_buffer(bool fp64, int64_t n, int PB, const int32_t *ids, const void *I, void *Buf, bool reset,
                         hipStream_t s);
