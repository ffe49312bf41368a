// One-workgroup FP64 CG for small two-mode systems (host interface).
#pragma once
#include "common.h"
#include "resident.h"

namespace cola {

constexpr int kSmallMax = 64;          // largest mode size of the one-workgroup FP64 path

struct SmallArgs {
    const ResSys* sys;       // per system: mode sizes, offsets into the FP64 factor / diagonal copies
    int32_t nitems;          // nsys * nrhs; item i = (system i / nrhs, right-hand side i % nrhs)
    int32_t nrhs;
    const double* fac64;
    const double* diag64;
    const double* B;         // packed right-hand sides
    double* X;               // packed solutions
    double tol;
    int32_t max_iters;
    int32_t x0_given;        // X holds the initial iterate (warm start); else x0 = 0
    cola_solve_info* info;   // one per item (system-major), or null
    ResHist rh;              // residual history, row = item (or empty)
};

// Whole FP64 CG solves (textbook recurrence, from x0 = 0 or the caller's X) of K1 (x) K2 + diag(d) + sigma2 I
// with both modes <= kSmallMax, one 1024-thread workgroup per item: the factors,
// the direction and the mode-2 product stay in LDS, x, r and the own part of p
// in registers, for every iteration.
hipError_t launch_small_cg64(const SmallArgs& a, hipStream_t s);

}  // namespace cola
