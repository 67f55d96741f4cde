// Internal launch tables: one per (degree, precision), filled by the
// per-degree translation units (dg_launch.hip compiled with DG_DEGREE=N).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

struct DgTable {
    hipError_t (*pack_star)(int64_t E, const double *dense, void *packed, hipStream_t s);
    hipError_t (*predictor)(int64_t E, double dt, const void *Q, const void *star, void *T, hipStream_t s);
    hipError_t (*time_integral)(int64_t E, double dt, const void *T, void *I, hipStream_t s);
    hipError_t (*volume)(int64_t E, const void *I, const void *star, void *Q, hipStream_t s);
    hipError_t (*local_flux)(int64_t E, const void *I, const double *Ap, void *Q, hipStream_t s);
    hipError_t (*neighbour_flux)(int64_t E, int64_t nI, const void *I, const int32_t *neigh, const uint8_t *fr,
                                 const double *Am, void *Q, hipStream_t s);
    hipError_t (*step_predict)(int64_t E, double dt, const void *Q, const void *star, void *I, void *traces,
                               hipStream_t s);
    hipError_t (*step_correct)(int64_t E, const void *I, const void *traces, const void *star, const double *Ap,
                               const double *Am, const int32_t *neigh, const uint8_t *fr, void *Q,
                               hipStream_t s);
};

void dg_table_2(DgTable *fp64, DgTable *fp32);
void dg_table_3(DgTable *fp64, DgTable *fp32);
void dg_table_4(DgTable *fp64, DgTable *fp32);
void dg_table_5(DgTable *fp64, DgTable *fp32);
void dg_table_6(DgTable *fp64, DgTable *fp32);
