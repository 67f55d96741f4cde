// Library-internal declarations shared by the C ABI translation units.
#pragma once
#include "dg.h"
#include "dg_tables.h"

// A compiled (degree, precision) configuration (opaque dg_plan of dg.h).
struct dg_plan {
    int degree;
    dg_precision prec;
    int B, Bf;
    DgTable tab;
};

// dg_step with its argument checks; debug_checks = false skips the
// synchronous neighbour-table validation (which copies the table to host
// memory).  The body of dg_step, shared with its variants.
int dg_step_impl(const dg_plan *plan, int64_t E, double dt, int n_steps, void *Q, void *I, void *traces,
                 void *traces_b, const void *star_packed, const double *Aplus, const double *Aminus,
                 const int32_t *neigh, const uint8_t *face_rot, hipStream_t s, bool debug_checks);

// Sets the calling thread's dg_last_error text; returns code.
int dg_set_error(int code, const char *msg);

// MADNESS contraction launcher (mra_kernels.hip).
hipError_t dg_mra_launch(bool fp64, int64_t nb, int p, int q, const void *S, const void *XL, const void *XR,
                         const void *YL, const void *YR, const void *ZL, const void *ZR, void *R, hipStream_t s);
