// Kronecker MVM of large two-mode operators in BF16 as two dense GEMMs.
//
// For A = sum_j U_j (x) V_j (+ diagonal) and X_r = p_r reshaped n1 x n2, the
// MVM is q_r = sum_j U_j X_r V_j^T: one product per mode, the cost of Table 2.
// When both modes are large the per-mode products are plain dense GEMMs with
// inner dimensions of 256 and more, so they are run as such on the BF16
// matrix cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation):
//
//   G1: T[(r, a'), (j, b)] = sum_b' P[(r, a'), b'] V_j[b, b']   (terms side by side in N)
//   G2: q_r[a, b] = sum_(j, a') U_j[a, a'] T_r[(j, a'), b]      (terms summed inside K)
//
// G1 stores T transposed per right-hand side (T_r[b][(j, a')]) so that both
// GEMMs take their operands k-contiguous.  Block tile 256 x 256, k slice 64,
// 8 waves (two per SIMD, so one wave's LDS and memory waits overlap the
// other's MFMAs) each owning 128 x 64 (4 x 2 MFMA tiles); two LDS stages, the
// next k slice copied from global memory straight into LDS while the current
// one is multiplied.  Block indices are mapped so that each XCD works on a
// contiguous group of tiles that share operand panels in its L2.
#include "gemm.h"

#include <algorithm>

#include "contract.h"

namespace cola {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = 256, BN = 256, KS = 64;
constexpr int kGT = 512;                         // threads of the GEMM kernels (8 waves)
constexpr int kStage = (BM + BN) * KS;           // bf16 elements of one LDS stage (A and B slices, 128-byte rows)
constexpr int kLdsBytes = 147456;                // two stages (131072 B) or the largest epilogue staging

__device__ inline floatx16 mfma32(bf16x8 a, bf16x8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Row of accumulator element v of a 32 x 32 MFMA tile held by `lane`; the
// column is lane % 32.
__device__ inline int row32(int lane, int v) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

// Tile index with all tiles of one XCD contiguous (blocks go to XCDs round robin).
__device__ inline int xcd_linear(int b, int T) {
    return (T % 8 == 0) ? (b % 8) * (T / 8) + b / 8 : b;
}

// One k slice: start the loads of the next slice into stage N and multiply
// the current one from stage S (A slice at the stage base, B slice
// 2 BM KS elements further, an offset that offb already holds).  The restrict
// qualifiers give the loads and the reads disjoint alias scopes, so the
// compiler does not wait for the loads in flight before reading the other
// stage.
__device__ __attribute__((always_inline)) inline void gemm_step(
    floatx16 (&acc)[4][2], const __bf16* __restrict__ S, __bf16* __restrict__ N, bool more, const __bf16* ga,
    int64_t lda, uint32_t aoff, const __bf16* gb, int64_t ldb, uint32_t boff, int wave, const uint32_t (&offa)[2][4],
    const uint32_t (&offb)[2][4]) {
    if (more) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int rb = 8 * q + wave;                   // row block of 8 rows
            __builtin_amdgcn_global_load_lds((const void*)(ga + (int64_t)rb * 8 * lda + aoff),
                                             (__attribute__((address_space(3))) void*)(N + rb * 8 * KS), 16, 0, 0);
            __builtin_amdgcn_global_load_lds((const void*)(gb + (int64_t)rb * 8 * ldb + boff),
                                             (__attribute__((address_space(3))) void*)(N + 2 * BM * KS + rb * 8 * KS),
                                             16, 0, 0);
        }
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        bf16x8 av[4], bv[2];
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i] = *(const bf16x8*)&S[i * 32 * KS + offa[i & 1][m]];
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) bv[jj] = *(const bf16x8*)&S[jj * 32 * KS + offb[jj & 1][m]];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int jj = 0; jj < 2; ++jj) acc[i][jj] = mfma32(av[i], bv[jj], acc[i][jj]);
    }
}

// acc += A_tile * B_tile^T over k in [0, nk) for this wave's 128 x 64 part.
// abase(k0) / bbase(k0) give the (block-uniform) address of row 0, column k0
// of the A / B tile; rows are lda / ldb elements apart and every row segment
// is 16-byte aligned.  Slices move from global memory straight into LDS
// (global_load_lds_dwordx4: lane l of a wave writes 16 bytes at LDS base +
// 16 l), one slice ahead of the one being multiplied, so no register staging
// and no LDS store instructions sit between the MFMAs.  LDS rows are 128
// bytes with no padding; 16-byte chunk c of row rho holds k chunk
// c ^ swz(rho), swz(rho) = (rho ^ rho / 8) % 8, which keeps the MFMA operand
// reads free of bank conflicts.  Wave w loads row blocks 8 w' + w (w' = 0..3)
// of 8 rows each; for those rows swz = (lane / 8) ^ w.
template <class ABase, class BBase>
__device__ inline void gemm_tile(floatx16 (&acc)[4][2], int nk, ABase abase, int64_t lda, BBase bbase, int64_t ldb,
                                 __bf16* smem) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) & 7;   // scalar, range known
    const int wm = wave >> 2, wn = wave & 3;
    // LDS: A slices of stages 0 and 1, then B slices of stages 0 and 1
    __bf16* const A0 = smem;
    __bf16* const A1 = smem + BM * KS;
    __bf16* const B0 = smem + 2 * BM * KS;
    const int lsw = ((lane >> 3) ^ wave) & 7;
    const uint32_t aoff = (uint32_t)((lane >> 3) * lda + 8 * ((lane & 7) ^ lsw));
    const uint32_t boff = (uint32_t)((lane >> 3) * ldb + 8 * ((lane & 7) ^ lsw));
    // Operand row rho = 32 t + (lane % 32) of a 32-row MFMA tile t, logical chunk
    // kc = 2 m + lane / 32 of k step m: swz = (lane % 8) ^ ((4 t + (lane % 32) / 8) % 8) depends on
    // t only through its parity, so eight per-lane offsets (parity x step) per operand serve every
    // tile and both stages; tiles add immediate offsets.
    uint32_t offa[2][4], offb[2][4];
#pragma unroll
    for (int par = 0; par < 2; ++par)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int sw = (lane & 7) ^ ((4 * par + ((lane & 31) >> 3)) & 7);
            const uint32_t o = (uint32_t)((lane & 31) * KS + 8 * ((2 * m + (lane >> 5)) ^ sw));
            offa[par][m] = o + (uint32_t)(wm * 128 * KS);
            offb[par][m] = o + (uint32_t)(2 * BM * KS + wn * 64 * KS);   // relative to the A base
        }
    {
        const __bf16* ga = abase(0);
        const __bf16* gb = bbase(0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int rb = 8 * q + wave;
            __builtin_amdgcn_global_load_lds((const void*)(ga + (int64_t)rb * 8 * lda + aoff),
                                             (__attribute__((address_space(3))) void*)(A0 + rb * 8 * KS), 16, 0, 0);
            __builtin_amdgcn_global_load_lds((const void*)(gb + (int64_t)rb * 8 * ldb + boff),
                                             (__attribute__((address_space(3))) void*)(B0 + rb * 8 * KS), 16, 0, 0);
        }
    }
    // stage pointers swap every slice; the restrict parameters of gemm_step
    // carry their disjointness to the compiler
    __bf16* cur = A0;
    __bf16* nxt = A1;
    for (int k0 = 0; k0 < nk; k0 += KS) {
        __builtin_amdgcn_s_waitcnt(0xF70);                 // vmcnt(0): this wave's part of slice k0 is in LDS
        __syncthreads();                                   // all of it; the other stage no longer read
        const bool more = k0 + KS < nk;
        const int kn = more ? k0 + KS : k0;
        gemm_step(acc, cur, nxt, more, abase(kn), lda, aoff, bbase(kn), ldb, boff, wave, offa, offb);
        __bf16* t = cur;
        cur = nxt;
        nxt = t;
    }
    __syncthreads();                                       // callers reuse the LDS for their epilogues
}

__device__ inline bool rhs_active(const Gemm2Args& a, int r) {
    return a.gate ? a.gate[(int64_t)r * a.gate_stride] != 0 : true;
}

// P16 = bf16(p) with p = r + beta p_old written back in FP32 (CG), or bf16(x).
template <bool CG>
__global__ __launch_bounds__(kThreads) void k_gemm2_pack(Gemm2Args a) {
    const int r = blockIdx.y;
    if (!rhs_active(a, r)) return;
    const int64_t n = (int64_t)a.n1 * a.n2;
    const double beta = CG ? a.cg[r].beta : 0.0;
    const float* X = a.X + (int64_t)r * n;
    const float* R = CG ? a.R + (int64_t)r * n : nullptr;
    float* P = CG ? a.P + (int64_t)r * n : nullptr;
    __bf16* P16 = a.P16 + (int64_t)r * n;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n / 8; i += (int64_t)gridDim.x * kThreads) {
        const int64_t e = i * 8;
        floatx4 x0 = *(const floatx4*)(X + e), x1 = *(const floatx4*)(X + e + 4);
        if constexpr (CG) {
            const floatx4 r0 = *(const floatx4*)(R + e), r1 = *(const floatx4*)(R + e + 4);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                x0[c] = pnew_of(r0[c], x0[c], beta);
                x1[c] = pnew_of(r1[c], x1[c], beta);
            }
            *(floatx4*)(P + e) = x0;
            *(floatx4*)(P + e + 4) = x1;
        }
        bf16x8 h;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            h[c] = (__bf16)x0[c];                          // round to nearest even
            h[c + 4] = (__bf16)x1[c];
        }
        *(bf16x8*)(P16 + e) = h;
    }
}

// G1: T_r[b][j n1 + a'] = sum_b' P16[r n1 + a', b'] V_j[b, b'].
__global__ __launch_bounds__(kGT) void k_gemm2_t(Gemm2Args a) {
    __shared__ __attribute__((aligned(16))) __bf16 smem[kLdsBytes / 2];
    const int Mt = a.nrhs * (a.n1 / BM), Nt = a.J * (a.n2 / BN);
    const int L = xcd_linear(blockIdx.x, Mt * Nt);
    int mt, nt;
    if (Mt % 4 == 0 && Nt % 8 == 0) {                      // 4 x 8 groups of tiles share A and B panels
        const int s = L / 32, w = L % 32, sn = Nt / 8;
        mt = (s / sn) * 4 + w / 8;
        nt = (s % sn) * 8 + w % 8;
    } else {
        mt = L / Nt;
        nt = L % Nt;
    }
    const int64_t m0 = (int64_t)mt * BM;
    const int r = (int)(m0 / a.n1), a0 = (int)(m0 % a.n1);
    if (!rhs_active(a, r)) return;
    const int n0 = nt * BN;
    const int j = n0 / a.n2, b0 = n0 % a.n2;
    const int64_t n2 = a.n2;
    const __bf16* Ab = a.P16 + m0 * n2;
    const __bf16* Bb = a.V + (int64_t)n0 * n2;
    floatx16 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) acc[i][jj] = floatx16{};
    gemm_tile(acc, a.n2, [&](int k0) { return Ab + k0; }, n2, [&](int k0) { return Bb + k0; }, n2, smem);

    // transposed bf16 store, one 32-column slice of the wave's sub-tile at a
    // time: FP32 staged in LDS as [column][row], then 8 rows per 16-byte store
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, wm = wave >> 2, wn = wave & 3;
    const int64_t ldt = (int64_t)a.J * a.n1;
    __bf16* Tb = a.T + ((int64_t)r * a.n2 + b0 + wn * 64) * ldt + (int64_t)j * a.n1 + a0 + wm * 128;
    constexpr int TP = 128 + 4;                            // staging pitch (floats)
    float* Ef = (float*)smem + wave * 32 * TP;             // [32 columns][128 rows]
#pragma unroll
    for (int jt = 0; jt < 2; ++jt) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int v = 0; v < 16; ++v) Ef[(lane & 31) * TP + i * 32 + row32(lane, v)] = acc[i][jt][v];
        __syncthreads();
#pragma unroll 2
        for (int c = 0; c < 8; ++c) {
            const int id = lane + 64 * c;
            const int col = id >> 4, m8 = (id & 15) * 8;
            const floatx4 lo = *(const floatx4*)&Ef[col * TP + m8];
            const floatx4 hi = *(const floatx4*)&Ef[col * TP + m8 + 4];
            bf16x8 h;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                h[u] = (__bf16)lo[u];                      // round to nearest even
                h[u + 4] = (__bf16)hi[u];
            }
            *(bf16x8*)(Tb + (int64_t)(jt * 32 + col) * ldt + m8) = h;
        }
        __syncthreads();
    }
}

// G2: q_r[a, b] = sum_(j, a') U_j[a, a'] T_r[b][j n1 + a'] + (sigma2 + d) p_r[a, b],
// with the CG epilogue's partial p.q and the step length alpha.
__global__ __launch_bounds__(kGT) void k_gemm2_y(Gemm2Args a) {
    __shared__ __attribute__((aligned(16))) __bf16 smem[kLdsBytes / 2];
    __shared__ double red[8];
    const int tn = a.n2 / BN, tpr = (a.n1 / BM) * tn;
    const int L = xcd_linear(blockIdx.x, a.nrhs * tpr);
    const int r = L / tpr, t = L % tpr;
    if (!rhs_active(a, r)) return;
    const int a0 = (t / tn) * BM, b0 = (t % tn) * BN;
    const int64_t n1 = a.n1, ldt = (int64_t)a.J * a.n1;
    const __bf16* Tr = a.T + ((int64_t)r * a.n2 + b0) * ldt;
    floatx16 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) acc[i][jj] = floatx16{};
    gemm_tile(acc, (int)ldt,
              [&](int k0) {
                  const int64_t j = k0 / n1;               // a 64-wide k slice never spans two terms
                  return a.U + j * n1 * n1 + a0 * n1 + (k0 - j * n1);
              },
              n1, [&](int k0) { return Tr + k0; }, ldt, smem);

    // epilogue, one 32-column slice of the wave's sub-tile at a time, staged in
    // LDS so that p, d and q move as 16-byte vectors along rows
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, wm = wave >> 2, wn = wave & 3;
    const int64_t n = n1 * a.n2;
    const bool cg = a.epi == EPI_CG;
    const float* Pr = (cg ? a.P : a.X) + (int64_t)r * n;
    float* Yr = a.Y + (int64_t)r * n;
    const float s2 = (float)a.sigma2;
    constexpr int FP = 32 + 4;                             // staging pitch (floats)
    float* Ef = (float*)smem + wave * 128 * FP;            // [128 rows][32 columns]
    // chunk c of slice jj: row c*8 + lane/8, columns (lane % 8)*4 .. +3 of the slice;
    // the lane part of the offset is fixed, the rest uniform
    const int64_t lane_e = (int64_t)(a0 + wm * 128 + (lane >> 3)) * a.n2 + b0 + wn * 64 + (lane & 7) * 4;
    auto e_of = [&](int jj, int c) -> int64_t { return lane_e + (int64_t)(8 * c) * a.n2 + jj * 32; };
    double dacc[4] = {0.0, 0.0, 0.0, 0.0};                 // p.q in FP64, four short chains
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int v = 0; v < 16; ++v) Ef[(i * 32 + row32(lane, v)) * FP + (lane & 31)] = acc[i][jj][v];
        __syncthreads();
#pragma unroll 4
        for (int c = 0; c < 16; ++c) {
            const int id = lane + 64 * c;
            const int row = id >> 3, c4 = (id & 7) * 4;
            const int64_t e = e_of(jj, c);
            const floatx4 y = *(const floatx4*)&Ef[row * FP + c4];
            const floatx4 p = *(const floatx4*)(Pr + e);
            floatx4 dg = floatx4{s2, s2, s2, s2};
            if (a.dvec) dg += *(const floatx4*)(a.dvec + e);
            floatx4 q;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                q[u] = y[u] + dg[u] * p[u];
                dacc[u] = __builtin_fma((double)p[u], (double)q[u], dacc[u]);
            }
            *(floatx4*)(Yr + e) = q;
        }
        __syncthreads();
    }
    const double dot = (dacc[0] + dacc[1]) + (dacc[2] + dacc[3]);
    if (!cg) return;
    const double s = block_sum8(dot, red);
    double tot;
    if (last_block_reduce8(s, a.partials + (int64_t)r * a.part_stride, a.counters + r, tpr, t, &tot, red) &&
        threadIdx.x == 0) {
        CgState& st = a.cg[r];
        if (!(tot > 0.0) || !finite_d(tot)) {
            st.status = finite_d(tot) ? COLA_ERR_NOT_SPD : COLA_ERR_NONFINITE;
            st.active = 0;
            atomicSub(&a.cnt->num_active, 1);
        } else {
            st.alpha = st.rho / tot;
        }
    }
}

}  // namespace

bool gemm2_supported(int prec, int Fv, const int64_t* dims) {
    return prec == COLA_PREC_BF16 && Fv == 2 && dims[0] >= BM && dims[1] >= BN && dims[0] % BM == 0 &&
           dims[1] % BN == 0;
}

int64_t gemm2_blocks_per_rhs(int64_t n1, int64_t n2) { return (n1 / BM) * (n2 / BN); }

hipError_t launch_gemm2(const Gemm2Args& a, int stage, hipStream_t s) {
    if (a.n1 % BM || a.n2 % BN || a.n1 < BM || a.n2 < BN || a.nrhs < 1 || a.J < 1) return hipErrorInvalidValue;
    const bool cg = a.epi == EPI_CG;
    if (cg && (!a.R || !a.P || !a.cg)) return hipErrorInvalidValue;
    if (stage == 0) {
        const int64_t n8 = (int64_t)a.n1 * a.n2 / 8;
        const int64_t bx = std::min<int64_t>(512, (n8 + kThreads - 1) / kThreads);
        dim3 grid((unsigned)bx, (unsigned)a.nrhs);
        if (cg) hipLaunchKernelGGL(k_gemm2_pack<true>, grid, dim3(kThreads), 0, s, a);
        else hipLaunchKernelGGL(k_gemm2_pack<false>, grid, dim3(kThreads), 0, s, a);
    } else if (stage == 1) {
        const int64_t T = (int64_t)a.nrhs * (a.n1 / BM) * a.J * (a.n2 / BN);
        hipLaunchKernelGGL(k_gemm2_t, dim3((unsigned)T), dim3(kGT), 0, s, a);
    } else {
        const int64_t T = (int64_t)a.nrhs * gemm2_blocks_per_rhs(a.n1, a.n2);
        hipLaunchKernelGGL(k_gemm2_y, dim3((unsigned)T), dim3(kGT), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace cola
