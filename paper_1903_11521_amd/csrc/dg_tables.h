// Internal launch tables: one per (degree, precision), filled by the
// per-degree translation units (dg_launch.hip and mfma_launch.hip compiled
// with DG_DEGREE=N).  Does not depend on the public header.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>


// Host image of one mesh of a (batched) time step; layout identical to the
// kernels' StepItem<real>.
struct DgItem {
    int64_t E;
    double dt;
    void *Q, *I, *traces;
    const void *star;
    const double *Ap, *Am;
    const int32_t *neigh;
    const uint8_t *face_rot;
    int64_t first_block;
    // neighbour index bound of the step corrector (>= E): indices in [E, nI)
    // name read-only face-trace slots after the item's own elements
    int64_t nI;
};

constexpr int DG_ELEMENTS_PER_BLOCK = 7;

struct DgTable {
    hipError_t (*pack_star)(int64_t E, const double *dense, void *packed, hipStream_t s);
    hipError_t (*predictor)(int64_t E, double dt, const void *Q, const void *star, void *T, hipStream_t s);
    hipError_t (*time_integral)(int64_t E, double dt, const void *T, void *I, hipStream_t s);
    hipError_t (*volume)(int64_t E, const void *I, const void *star, void *Q, hipStream_t s);
    hipError_t (*local_flux)(int64_t E, const void *I, const double *Ap, void *Q, hipStream_t s);
    hipError_t (*neighbour_flux)(int64_t E, int64_t nI, const void *I, const int32_t *neigh, const uint8_t *fr,
                                 const double *Am, void *Q, hipStream_t s);
    hipError_t (*step_predict)(const DgItem &it, hipStream_t s);
    hipError_t (*step_correct)(const DgItem &it, hipStream_t s);
    // corrector of one step and predictor of the next in one launch: reads the
    // traces in it.traces, writes the next step's traces to tr_out
    hipError_t (*step_fused)(const DgItem &it, void *tr_out, hipStream_t s);
    // whether the fused launch is used (it is faster than the two separate
    // launches only at low degree; measured on MI355X, all precisions)
    bool fuse_step;
    // batched: items (device array) of one degree; block_item maps each of the
    // nblocks workgroups to its item
    hipError_t (*batch_predict)(const DgItem *items, const int32_t *block_item, int64_t nblocks, hipStream_t s);
    hipError_t (*batch_correct)(const DgItem *items, const int32_t *block_item, int64_t nblocks, hipStream_t s);
    // fused simulations (16 per element, DOFs [E][9][B][16]): the two step
    // launches; null where the precision has no fused form
    hipError_t (*fused_predict)(const DgItem &it, hipStream_t s);
    hipError_t (*fused_correct)(const DgItem &it, hipStream_t s);
};

// tables for DG_FP64, DG_FP32 and DG_MIXED (dg_launch.hip)
void dg_table_2(DgTable *fp64, DgTable *fp32, DgTable *mixed);
void dg_table_3(DgTable *fp64, DgTable *fp32, DgTable *mixed);
void dg_table_4(DgTable *fp64, DgTable *fp32, DgTable *mixed);
void dg_table_5(DgTable *fp64, DgTable *fp32, DgTable *mixed);
void dg_table_6(DgTable *fp64, DgTable *fp32, DgTable *mixed);
// tables for DG_BF16X3 (mfma_launch.hip); entries the form does not
// implement are null
void dg_mtable_2(DgTable *t);
void dg_mtable_3(DgTable *t);
void dg_mtable_4(DgTable *t);
void dg_mtable_5(DgTable *t);
void dg_mtable_6(DgTable *t);

