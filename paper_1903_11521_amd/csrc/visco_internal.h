// Viscoelastic step kernels (visco_kernels.hip), used by visco.cpp and the
// batch in dg_api.cpp.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// One viscoelastic mesh of a launch.  Elements of all items of a launch form
// one work list; `first` is the item's offset in it (items sorted by first).
struct VItem {
    int64_t E;
    int64_t first;
    double dt;
    double omega[3];              // relaxation frequencies of the three mechanisms
    double *Q, *I, *traces;       // [E][27][B], [E][27][B], [E][4][9][Bf]
    const double *star;           // [E][3][27][9]
    const double *Ap, *Am;        // [E][4][27][9]
    const int32_t *neigh;         // [E][4], local to the item
    const uint8_t *face_rot;      // [E][4]
};

// One time step: predictor (derivatives, time integral, face traces) then
// corrector over every element of the work list.  items: device array of
// n_items entries, or null with `one` describing the single item; total:
// elements in the work list; blob: the degree's reference matrices on the
// device.
hipError_t visco_step_launch(int degree, const VItem *items, int n_items, const VItem &one, int64_t total,
                             const double *blob, hipStream_t s);

// Launch shape of a degree: waves per workgroup (4 or 8) and resident
// workgroups per CU of the persistent grids (0: as many as fit).  Process-wide,
// set by dg_visco_tune; the default is 4 waves (8 at degree 6), all that fit.
struct VShape {
    int waves;
    int per_cu;
};
VShape visco_shape(int degree);
void visco_set_shape(int degree, VShape shape);

// Sets the kernels' LDS limits and reads their occupancy for a degree and
// wave count (done by the first launch otherwise; call before recording
// launches into a graph).  max_per_cu (may be null): the larger of the two
// kernels' resident workgroups per CU.
hipError_t visco_prepare_shape(int degree, int waves, int *max_per_cu);
hipError_t visco_prepare(int degree);

// visco_step_launch with an explicit shape.
hipError_t visco_step_shape(int degree, VShape shape, const VItem *items, int n_items, const VItem &one,
                            int64_t total, const double *blob, hipStream_t s);
