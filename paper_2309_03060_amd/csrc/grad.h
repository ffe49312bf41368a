// Adjoint-gradient contractions and the tile autotuner (host launchers).
#pragma once
#include "op.h"

namespace cola {

// Factor, diagonal and sigma2 gradients of one system from X and Lambda = A^{-1} G, times `scale`
// (1 for the solve VJP; -1/N for the Hutchinson estimate of the log det gradient over N probes).
int32_t grad_system(cola_op_s* op, const SysInfo& s, const double* X, const double* Lam, int nrhs,
                    void* const* dfactors, void* ddiag, double* dsigma2, hipStream_t st, double scale = 1.0);

// Time every tile candidate of every contraction pass of this op at nrhs.
int32_t autotune_op(cola_op_s* op, int nrhs, hipStream_t st);

// Enqueue the mode products of one term's factors on X, skipping mode `skip`
// (-1: none); output in `out` (workspace-sized).  FP64.
int32_t apply_modes_f64(cola_op_s* op, const SysInfo& s, int term, int skip, const double* X, int nrhs,
                        double* out, hipStream_t st);

}  // namespace cola
