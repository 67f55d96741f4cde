// Viscoelastic step launcher (visco_kernels.hip), used by visco.cpp.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// relaxation frequencies of the three mechanisms (kernel argument by value)
struct VOmega {
    double w[3];
};

hipError_t visco_step_launch(int degree, int64_t E, double dt, double *Q, double *I, double *traces,
                             const double *star, const double *Ap, const double *Am, const int32_t *neigh,
                             const uint8_t *face_rot, VOmega om, const double *blob, hipStream_t s);
