// Symmetric eigendecomposition of Kronecker factors and the eigenvalue scaling
// of the Kronecker-eigen solve (host interface).
#pragma once
#include "common.h"

namespace cola {

// One-sided (Hestenes) Jacobi on a symmetric positive semi-definite n x n
// matrix A (FP64, row-major; by symmetry also column-major).  On return
// V (column-major, column j = eigenvector j; equivalently row-major V^T) and
// lam[j] = ||A v_j|| = the j-th eigenvalue.  `work` holds n*n doubles, `off`
// one double (largest relative off-diagonal measure of the last sweep).
// Synchronises the stream once per sweep to test convergence.
int32_t jacobi_eig(const double* A, int64_t n, double* V, double* lam, double* work, double* off,
                   double tol, int max_sweeps, hipStream_t s);

// Z[r, i1, i2, i3] = Y[r, i1, i2, i3] / (lam1[i1] lam2[i2] lam3[i3] + sigma2) for
// nrhs packed right-hand sides of one system (F modes, unused dims = 1).
hipError_t eig_scale(const double* Y, double* Z, int64_t nrhs, int F, const int64_t* dims,
                     const double* const* lam, double sigma2, hipStream_t s);

// out = in^T for an n x n FP64 matrix.
hipError_t transpose_f64(const double* in, double* out, int64_t n, hipStream_t s);

}  // namespace cola
