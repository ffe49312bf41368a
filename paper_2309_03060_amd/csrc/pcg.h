// Exact operator diagonals, preconditioned-CG vector kernels and probe
// diagonal estimators (host interface).
#pragma once
#include "common.h"

namespace cola {

// One system's operator sum_j K_j1 (x) .. (x) K_jF + diag(d) + sigma2 I as plain
// pointers: mode k's factor of term j is fac[k] + j * dims[k]^2 (row-major).
struct DiagArgs {
    int32_t J;
    int32_t F;               // modes (unused trailing dims are 1)
    int64_t dims[3];
    const double* fac[3];
    const double* dvec;      // n entries, or null
    double sigma2;
    int64_t n;
};

// out[i] = Diag(A)[i], or 1 / Diag(A)[i] when invert (row-major multi-index).
hipError_t kron_diagonal(const DiagArgs& a, double* out, bool invert, hipStream_t s);

// *out = Tr(A - first term) / n = sigma2 + mean(d) + sum_{j >= 1} prod_k mean(Diag(K_jk)).
hipError_t trace_shift(const DiagArgs& a, double* out, hipStream_t s);

// x += alpha p, r -= alpha q for the active right-hand sides; the last block of
// each sums r.r, counts the iteration and decides convergence (r.r <= tol2),
// the iteration limit or non-finite values, as plain CG does; rh records the
// residual history (or is empty).
hipError_t pcg_update(double* x, double* r, const double* p, const double* q, int64_t n, int nrhs, CgState* cg,
                      double* partials, int part_stride, uint32_t* counters, SolveCounters* cnt, int max_blocks,
                      hipStream_t s, ResHist rh = ResHist{});

// z = dinv . r when dinv is given (else z already holds M^{-1} r); rho' = r.z,
// beta = rho' / rho, rho = rho' for the active right-hand sides; rho' <= 0 or
// non-finite stops the right-hand side (M not positive definite).
hipError_t pcg_precond_dot(const double* r, double* z, const double* dinv, int64_t n, int nrhs, CgState* cg,
                           double* partials, int part_stride, uint32_t* counters, SolveCounters* cnt,
                           int max_blocks, hipStream_t s);

// After a preconditioned solve: rho = r.r (kept in rho_true by pcg_update) so the
// solve info reports ||b - A x|| / ||b|| as for plain CG.
hipError_t pcg_finish(CgState* cg, int nrhs, hipStream_t s);

// out[i] (+)= scale * sum_j Z[j][i] * Q[j][i] over nprobes vectors of n entries.
hipError_t probe_accumulate(const double* Z, const double* Q, int64_t n, int nprobes, double scale, double* out,
                            bool accumulate, hipStream_t s);

}  // namespace cola
