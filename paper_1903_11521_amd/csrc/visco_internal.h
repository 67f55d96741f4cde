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

// Sets the kernels' LDS limits and persistent grid sizes for a degree (done
// by the first launch otherwise; call before recording launches into a graph).
hipError_t visco_prepare(int degree);
