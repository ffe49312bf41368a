// Resident batched CG for many small two-mode systems (host interface).
#pragma once
#include "common.h"

namespace cola {

// Per-system geometry for the resident kernels (device memory).
struct ResSys {
    int32_t n1, n2;        // mode sizes (<= kResMax)
    int64_t n;             // n1 * n2
    int64_t vec_off;       // unknowns of earlier systems (packed offset = nrhs * vec_off + rhs * n)
    int64_t k1_off, k2_off;// factor offsets (same in the FP32 and FP64 copies)
    int64_t diag_off;      // -1: no diagonal vector
    double sigma2;
};

struct ResArgs {
    const ResSys* sys;
    const int32_t* order;  // work-queue order of items (largest systems first)
    int32_t nitems;        // nsys * nrhs; item i = (system i / nrhs, rhs i % nrhs)
    int32_t nrhs;
    uint32_t* queue;       // work counter, zero at launch
    const float* fac32;
    const double* fac64;
    const float* diag32;
    const double* diag64;
    float* x; float* r; float* p;   // packed FP32 CG state
    double* x64;                    // packed FP64 solution
    const double* b64;              // packed FP64 right-hand sides
    double* t64;                    // packed FP64 scratch (residual intermediate)
    CgState* st;                    // per item
    SolveCounters* cnt;
    int32_t all_items;              // residual kernel: final pass (items without a certified residual)
};

constexpr int kResMax = 128;        // largest mode size handled by the resident kernel

hipError_t launch_resident_prepare(const ResArgs& a, double tol, int max_iters, double delta, hipStream_t s);
hipError_t launch_resident_cg(const ResArgs& a, int grid, hipStream_t s);
hipError_t launch_resident_resid64(const ResArgs& a, hipStream_t s);
hipError_t launch_resident_info(const ResArgs& a, cola_solve_info* info, hipStream_t s);

}  // namespace cola
