// Stochastic Lanczos quadrature of log det A from recorded CG coefficients (host interface).
#pragma once
#include "common.h"

namespace cola {

constexpr size_t kSlqLds = 61440;       // LDS per block for the per-probe tridiagonal scratch

// Probes handled per block for tridiagonals of up to hist_len rows (0: too long).
int slq_threads_per_block(int hist_len);

// For each probe g: est[g] = ||z_g||^2 e1^T log(T_g) e1, with T_g built from the
// (alpha, beta) pairs hist[g * 2 * hist_len ...] of its cg[g].iters iterations
// (NaN after a CG breakdown); then *logdet = the mean of est (one device double).
hipError_t slq_logdet(const double* hist, int hist_len, const CgState* cg, int nprobes, double* est,
                      double* logdet, hipStream_t s);

}  // namespace cola
