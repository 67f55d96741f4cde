// Host-side generator of the reference matrices (see refmat.cpp).
#pragma once
#include <cstddef>

namespace dgref {
int basis_size(int N);
int face_basis_size(int N);
// Number of doubles in the blob written by build():
//   Khat[3][B][B], Ktilde[3][B][B], R[4][B][Bf], Rhat[4][B][Bf], f[3][Bf][Bf],
//   mass[B], face_mass[Bf]   (row-major)
size_t blob_size(int N);
int build(int N, double *out);
void gauss_jacobi(int n, double alpha, double *x, double *w);
}  // namespace dgref
