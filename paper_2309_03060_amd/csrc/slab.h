// Fused mode-2/mode-3 slab product (host launcher).
#pragma once
#include "common.h"

namespace cola {

struct SlabArgs {
    int64_t nslabs;        // nrhs * n1 slabs of n2 x n3
    int64_t a_per_rhs;     // slabs per right-hand side (n1)
    int32_t n2, n3;
    int32_t nterms;        // one output per term (grid dimension)
    int32_t pnew;          // slab = R + beta * X (first pass of a CG iteration)
    const void* X;
    const void* R;
    void* Y; int64_t y_tstride;
    const void* K2; const void* K3; int64_t k2_tstride, k3_tstride;
    const int32_t* gate; int32_t gate_stride;   // per-RHS flag; null: no gating
    CgState* cg;                                // beta of the direction update
};

bool slab_supported(int prec, int64_t n2, int64_t n3);
hipError_t launch_slab23(int prec, const SlabArgs& a, hipStream_t s);

}  // namespace cola
