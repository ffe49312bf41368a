// Persistent fused CG for one-term three-mode FP32 operators with 64-wide
// modes (host interface).
#pragma once
#include "common.h"

namespace cola {

// One launch runs up to `iters` CG iterations for `nrhs` right-hand sides of
// one system K1 (x) K2 (x) K3 + diag(d) + sigma2 I with n = 64^3.  Every
// right-hand side is owned by a group of `bpr` co-resident blocks that meet at
// group barriers; the state machine is the one of the separate-kernel path
// (direction, MVM, step length, update, convergence and reliable-update test).
struct FusedCgArgs {
    int32_t nrhs;        // right-hand sides of this launch, one block group each
    int32_t bpr;         // blocks per right-hand side: 8 or 16
    int32_t iters;       // iterations to run; a right-hand side leaves once inactive
    const float* K1; const float* K2; const float* K3;   // 64 x 64, row-major
    const float* dvec;   // diagonal, n entries, or null
    double sigma2;
    float* x; float* r; float* p;   // right-hand side g at offset g * n
    float* T;            // intermediate (K2, K3 product), same layout
    CgState* cg;         // right-hand side g at cg[g]
    double* slots;       // 3 * nrhs * bpr barrier slots, all bits set at launch
    uint32_t* err;       // set to 1 when a barrier wait times out
    SolveCounters* cnt;
};

bool fused_cg_supported(int prec, int Fv, int J, const int64_t* dims);

// Largest number of fused-CG blocks that can be resident at once on the
// current device (0 when cooperative launches are unavailable).
int fused_cg_max_blocks();

// Blocks per right-hand side for a solve of nrhs right-hand sides.
int fused_cg_blocks_per_rhs(int nrhs, int max_blocks);

// Cooperative launch of nrhs * bpr blocks (nrhs * bpr <= fused_cg_max_blocks()).
hipError_t launch_fused_cg(const FusedCgArgs& a, hipStream_t s);

// After the launches of a solve enqueued without host checks: if a group barrier
// timed out (*err set), every right-hand side of the solve is reported as
// COLA_ERR_HIP and stops (the launch's results are void).
hipError_t fused_cg_report_timeout(const uint32_t* err, CgState* cg, int nrhs, hipStream_t s);

}  // namespace cola
