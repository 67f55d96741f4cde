// Launchers of the local-time-stepping kernels (lts_kernels.hip), used by
// the scheduler in lts.cpp.  A face-trace slot holds an element's 4 face
// blocks of 9 Bf values (the layout of dg_step's trace array); TB is its
// length in values.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Ghost slots of one cluster: for ghost g (neighbour v = ids[g] in another
// cluster), dst[g] =
//   kind 1 (one cluster up), half 0:  half_tr[v]                (first half of v's step)
//   kind 1,                  half 1:  up_tr[v] - half_tr[v]     (second half)
//   kind 2 (one cluster down):         buf_tr[v]                (v's two step traces summed)
hipError_t dg_lts_ghosts(bool fp64, int64_t n, int TB, const int32_t *ids, const int8_t *kind, int half,
                         const void *up_tr, const void *half_tr, const void *buf_tr, void *dst, hipStream_t s);
// buf_tr[v] = src_tr[v] (reset) or buf_tr[v] + src_tr[v] for v = ids[j].
hipError_t dg_lts_tbuffer(bool fp64, int64_t n, int TB, const int32_t *ids, const void *src_tr, void *buf_tr,
                          bool reset, hipStream_t s);
