// LinA (ADER-DG-SEM on cuboids): internal declarations shared by lina.cpp
// and lina_kernels.hip.  Coefficient blob of order O (all of the step's
// precision on the device): Kt [O][O], Kh [O][O], w [O], star [3][4][4],
// Ap [6][4][4], Am [6][4][4].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// fills the FP64 blob of order O (host)
int lina_blob(int O, double rho0, double K0, double h, double *out);
// one step: predictor + weak derivatives + sides, then the side fluxes
hipError_t lina_launch(bool fp64, int O, int64_t E, double dt, void *Q, void *sides, const void *coef,
                       const int32_t *neigh, hipStream_t s);
