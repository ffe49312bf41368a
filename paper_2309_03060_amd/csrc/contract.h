// Mode contraction pass of the Kronecker MVM: host-visible argument block.
#pragma once
#include "common.h"

namespace cola {

enum Epilogue : int32_t {
    EPI_STORE  = 0,   // Y = contraction
    EPI_CG     = 1,   // p = r + beta p_old (written back), q = contraction + diag * p, mu partial p.q
    EPI_RESID  = 2,   // r = b - (contraction + diag * x), partial r.r
    EPI_MATVEC = 3,   // y = contraction + diag * x
    EPI_RESID_CG = 4, // as EPI_RESID, total ||r||^2 goes to CgState::rho_true (reliable updates)
};

// One pass contracts a single tensor mode with one factor per Kronecker term.
//
// ROWS layout (last mode, inner extent 1):  Y[g, i]    = sum_l K[i, l] X[g, l]
// COLS layout (other modes):                Y[g, i, b] = sum_l K[i, l] X[g, l, b]
// where g runs over (right-hand side, leading modes) and b over trailing modes.
struct PassArgs {
    int64_t G;           // batches (COLS) or rows (ROWS)
    int64_t B;           // inner extent (COLS); 1 for ROWS
    int32_t nk;          // size of the contracted mode
    int32_t nsum;        // terms summed inside the K loop (last pass of a sum of terms)
    int32_t nout;        // terms with separate outputs (earlier passes)
    int32_t pnew;        // 1: vector operand = R + beta * X (first pass of a CG iteration)
    int64_t a_per_rhs;   // batches (COLS) / rows (ROWS) per right-hand side

    const void* X; int64_t x_tstride;   // input, element stride between terms
    void* Y;       int64_t y_tstride;   // output
    const void* K; int64_t k_tstride;   // factor of this mode for term t at K + t*k_tstride
    int64_t k_plane;                    // BF16x3: element offset between the three split planes
    const void* R;                      // residual for the pnew prologue

    int32_t epi;          // Epilogue
    const void* Ep;       // CG: p_old;  RESID / MATVEC: x
    const void* Er;       // CG: r;      RESID: b
    void* Epout;          // CG: p_new
    void* Ex;             // CG: the iterate, when the first pass may apply x += alpha p_old (else null)
    void* Ep2;            // CG with Ex: a second direction buffer an engine may alternate with Epout
                          // (pbuf / pswap of the CG state), else null
    const void* dvec;     // diagonal d (vector element type), may be null
    double sigma2;

    double* partials; int32_t part_stride;   // per right-hand side
    uint32_t* counters;                       // per right-hand side
    const int32_t* gate; int32_t gate_stride; // per-RHS flag (int32 stride); null: no gating
    CgState* cg;                              // CG scalars (beta, alpha, finalize)
    OuterState* outer;                        // refinement residual finalize
    SolveCounters* cnt;
};

struct TileCfg { int wm, wn; };   // MFMA 16x16 tiles per wave; block tile is (32*wm) x (32*wn)

// Launch one pass; `prec` is COLA_PREC_*, `rows` selects the ROWS layout.
hipError_t launch_contract(int prec, bool rows, const PassArgs& a, TileCfg cfg, hipStream_t s);

// Blocks per right-hand side of a COLS pass (for sizing reduction partials).
int64_t contract_blocks_per_g(int prec, const PassArgs& a, TileCfg cfg);

}  // namespace cola
