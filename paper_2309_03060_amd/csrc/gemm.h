// Kronecker MVM of large two-mode operators in BF16 as two dense GEMMs (host interface).
#pragma once
#include "common.h"

namespace cola {

// A = sum_j U_j (x) V_j + diag(d) + sigma2 I with n1 x n1 factors U_j and
// n2 x n2 factors V_j, both mode sizes multiples of 256.  One MVM q = A p is
//   pack : P16 = bf16(p)  (CG: p = r + beta p_old first, written back in FP32)
//   G1   : T[(r, a'), (j, b)] = sum_b' P16[(r, a'), b'] V_j[b, b']    (all terms at once)
//   G2   : q_r[a, b] = sum_(j, a') U_j[a, a'] T_r[(j, a'), b] + (sigma2 + d) p_r[a, b]
// G1 stores T transposed per right-hand side, T_r[b][(j, a')], so both GEMMs
// read their operands k-contiguous; G2 sums the terms inside its k loop.
struct Gemm2Args {
    int32_t n1, n2, J, nrhs;
    const __bf16* U;          // term j's mode-1 factor at U + j * n1 * n1 (row-major)
    const __bf16* V;          // term j's mode-2 factor at V + j * n2 * n2
    const float* X;           // CG: p_old; matvec: x
    const float* R;           // CG: r; matvec: null
    float* P;                 // CG: p_new (may alias X); matvec: null
    __bf16* P16;              // nrhs * n1 * n2
    __bf16* T;                // nrhs * n2 * J * n1
    float* Y;                 // q
    const float* dvec;        // n1 * n2 or null
    double sigma2;
    int32_t epi;              // EPI_CG or EPI_MATVEC
    CgState* cg;
    const int32_t* gate; int32_t gate_stride;
    double* partials; int32_t part_stride;
    uint32_t* counters;
    SolveCounters* cnt;
};

bool gemm2_supported(int prec, int Fv, const int64_t* dims);

// Enqueue the three kernels of one MVM.  Each is timed under its own profile
// class by the caller: `stage` 0 = pack, 1 = G1, 2 = G2.
hipError_t launch_gemm2(const Gemm2Args& a, int stage, hipStream_t s);

// Blocks per right-hand side of G2 (reduction partials needed).
int64_t gemm2_blocks_per_rhs(int64_t n1, int64_t n2);

// The same two GEMMs in FP64 (v_mfma_f64_16x16x4f64) with the FP64 master
// factors, for the FP64 passes of two-mode operators whose modes are
// multiples of 256: the residuals b - A x of mixed-precision solves, FP64 CG
// and FP64 products.
//   pack (CG): p = r + beta p_old, written in place of p_old
//   G1: T_r[b][(j, a')] = sum_b' X[(r, a'), b'] V_j[b, b']
//   G2: y_r[a, b] = sum_(j, a') U_j[a, a'] T_r[b][(j, a')], then the epilogue
//       (EPI_MATVEC: y + (sigma2 + d) x; EPI_CG: q = y + (sigma2 + d) p, p.q and
//       the step length; EPI_RESID / EPI_RESID_CG: b - (y + (sigma2 + d) x) and
//       its squared norm).
struct Gemm64Args {
    int32_t n1, n2, J, nrhs;
    const double* U;          // term j's mode-1 factor at U + j * n1 * n1
    const double* V;          // term j's mode-2 factor at V + j * n2 * n2
    const double* X;          // G1 operand: x, or p (CG, after the pack pass)
    const double* R;          // CG: r
    const double* Pold;       // CG: p_old
    double* P;                // CG: p_new (may alias Pold)
    double* T;                // nrhs * n2 * J * n1
    double* Y;                // output
    const double* Ep;         // epilogue operand: x, or p_new (CG)
    const double* Er;         // residual epilogues: b
    const double* dvec;       // n1 * n2 or null
    double sigma2;
    int32_t epi;
    CgState* cg;
    OuterState* outer;
    const int32_t* gate; int32_t gate_stride;
    double* partials; int32_t part_stride;
    uint32_t* counters;
    SolveCounters* cnt;
};

bool gemm64_supported(int Fv, const int64_t* dims);

// `stage` 0 = pack (CG only), 1 = G1, 2 = G2.
hipError_t launch_gemm64(const Gemm64Args& a, int stage, hipStream_t s);

// Blocks per right-hand side of the FP64 G2.
int64_t gemm64_blocks_per_rhs(int64_t n1, int64_t n2);

// One-term three-mode operators with every mode a multiple of 256 in FP64: three passes of the
// G1 kernel (J = 1), each contracting the contiguous mode of its input and storing its output
// new mode first (n1 = rows per right-hand side of the pass's input, n2 = its mode size); the
// last pass (`final`) carries the epilogue of G2 and writes Y in the original layout.  The pack
// pass of CG is launch_gemm64 stage 0 with n1 * n2 = n.
bool gemm64_3_supported(int Fv, int J, const int64_t* dims);
int64_t gemm64_3_blocks_per_rhs(int64_t n1, int64_t n2, int64_t n3);
hipError_t launch_gemm64_pass(const Gemm64Args& a, bool final, hipStream_t s);

}  // namespace cola
