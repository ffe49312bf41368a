// Kronecker MVM of three-mode FP32 operators with 256-wide modes as three dense GEMMs (host interface).
#pragma once
#include "common.h"

namespace cola {

// One term K1 (x) K2 (x) K3 (+ diagonal + sigma2 I), n1, n2 multiples of 256
// and n3 = 256, in FP32 or BF16x3 working precision.  Each pass multiplies the last (contiguous) mode of its input
// by its factor and stores the result with the new mode first, so the next
// pass again finds its mode contiguous:
//   pass 3: Z1[r][c'][a][b] = sum_c  P[r][a][b][c]  K3[c', c]   (P = r + beta p_old when CG)
//   pass 2: Z2[r][b'][c'][a] = sum_b  Z1[r][c'][a][b] K2[b', b]
//   pass 1: q [r][a'][b'][c'] = sum_a Z2[r][b'][c'][a] K1[a', a] (+ diagonal; CG epilogue)
struct Gemm3Args {
    int32_t n1, n2, n3, nrhs;
    int32_t bf16x3;           // 0: FP32 MFMA; 1: BF16x3 (both operands split three ways when staged)
    const float* K1; const float* K2; const float* K3;   // FP32 working copies of the factors
    const float* X;           // CG: p_old (p_new is written back in place); matvec: x
    const float* R;           // CG: r
    float* Xit;               // CG with reliable updates: the iterate; the first pass applies the
                              // previous step's x += alpha p_old (deferred from the update), else null
    float* P2;                // BF16x3 CG with Xit, all modes 256: second direction buffer.  The first
                              // pass reads p_old from buffer pbuf and writes p_new to the other one;
                              // the middle and last passes take x += alpha p_old (half of x each)
    float* Z1; float* Z2;     // intermediates, nrhs * n1 * n2 * n3 each
    float* Y;                 // q
    const float* dvec;        // n or null
    double sigma2;
    int32_t epi;              // EPI_CG or EPI_MATVEC
    CgState* cg;
    const int32_t* gate; int32_t gate_stride;
    double* partials; int32_t part_stride;
    uint32_t* counters;
    SolveCounters* cnt;
};

bool gemm3_supported(int prec, int Fv, int J, const int64_t* dims);

// Tile edge of the engine (n3 always equals it); the double-buffered direction of the BF16x3
// engine needs every mode equal to it.
constexpr int kGemm3Tile = 256;

// Enqueue one pass: mode 3, 2 or 1 (in that order).
hipError_t launch_gemm3(const Gemm3Args& a, int mode, hipStream_t s);

}  // namespace cola
