// Stochastic Lanczos quadrature of log det A from recorded CG coefficients (host interface).
#pragma once
#include "common.h"

namespace cola {

constexpr int kSlqMaxSteps = 2048;      // longest tridiagonal (CG steps per probe) held in LDS

// For each probe g: est[g] = ||z_g||^2 e1^T log(T_g) e1, with T_g built from the
// (alpha, beta) pairs hist[g * 2 * hist_len ...] of its cg[g].iters iterations
// (NaN after a CG breakdown); then *logdet = the mean of est (one device double).
// hist_len <= kSlqMaxSteps.
hipError_t slq_logdet(const double* hist, int hist_len, const CgState* cg, int nprobes, double* est,
                      double* logdet, hipStream_t s);

}  // namespace cola
