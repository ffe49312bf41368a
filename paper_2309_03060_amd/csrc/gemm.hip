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


// ---------------------------------------------------------------------------
// FP64 engine.  Block tile 256 (A rows) x 128 (B rows), k slice 16, 8 waves
// (two per SIMD) each owning 64 x 64 (4 x 4 tiles of v_mfma_f64_16x16x4f64,
// whose A operand lane l holds row l % 16, k l / 16, and whose accumulator
// element v of lane l is row 4 v + l / 16, column l % 16).  Slices move from
// global memory straight into one of two LDS stages (global_load_lds_dwordx4)
// one slice ahead of the one being multiplied.  LDS rows are 128 bytes (A rows
// 0..255, then B rows 256..383); 16-byte chunk c of row rho sits at chunk
// c ^ h(rho), h(rho) = (rho / 2) % 8, which puts the 32 lanes of each half of a
// fragment read (16 rows, two k) on 64 distinct banks.

constexpr int DM = 256, DN = 128, DKS = 16;
constexpr int kDStage = (DM + DN) * DKS * 8;          // bytes of one stage (48 KiB)

__device__ inline doublex4 mfma64(double a, double b, doublex4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Issue the copies of one k slice: A rows from ga (row stride lda), B rows from
// gb (stride ldb), into stage N.  Wave w copies row blocks 8 q + w of 8 rows.
__device__ __attribute__((always_inline)) inline void g64_issue(char* __restrict__ N, const double* ga, int64_t lda,
                                                               const double* gb, int64_t ldb, int64_t aoff,
                                                               int64_t boff, int wave) {
#pragma unroll
    for (int q = 0; q < DM / 64; ++q) {
        const int rb = 8 * q + wave;
        __builtin_amdgcn_global_load_lds((const void*)(ga + (int64_t)rb * 8 * lda + aoff),
                                         (__attribute__((address_space(3))) void*)(N + rb * 8 * 128), 16, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < DN / 64; ++q) {
        const int rb = 8 * q + wave;
        __builtin_amdgcn_global_load_lds((const void*)(gb + (int64_t)rb * 8 * ldb + boff),
                                         (__attribute__((address_space(3))) void*)(N + (DM + rb * 8) * 128), 16, 0,
                                         0);
    }
}

__device__ __attribute__((always_inline)) inline void g64_step(doublex4 (&acc)[4][4], const char* __restrict__ S,
                                                              char* __restrict__ N, bool more, const double* ga,
                                                              int64_t lda, const double* gb, int64_t ldb,
                                                              int64_t aoff, int64_t boff, int wave,
                                                              const uint32_t (&fo)[4], uint32_t abyte,
                                                              uint32_t bbyte) {
    if (more) g64_issue(N, ga, lda, gb, ldb, aoff, boff, wave);
#pragma unroll
    for (int m = 0; m < DKS / 4; ++m) {
        double av[4], bv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i] = *(const double*)(S + abyte + i * 16 * 128 + fo[m]);
#pragma unroll
        for (int j = 0; j < 4; ++j) bv[j] = *(const double*)(S + bbyte + j * 16 * 128 + fo[m]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = mfma64(av[i], bv[j], acc[i][j]);
    }
}

// acc += A_tile * B_tile^T over k in [0, nk): abase(k0) / bbase(k0) give row 0, column k0 of
// the A / B tile (rows lda / ldb elements apart, 16-byte aligned).
template <class ABase, class BBase>
__device__ inline void gemm64_tile(doublex4 (&acc)[4][4], int nk, ABase abase, int64_t lda, BBase bbase,
                                   int64_t ldb, char* smem) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) & 7;   // scalar, range known
    const int wa = wave >> 1, wb = wave & 1;
    // copies: lane l fills row rb*8 + l/8, physical chunk l % 8, i.e. logical chunk (l % 8) ^ h with
    // h = 4 (rb % 2) + l / 16 = 4 (w % 2) + l / 16 for this wave's row blocks
    const int lc = (lane & 7) ^ (4 * (wave & 1) + (lane >> 4));
    const int64_t aoff = (int64_t)(lane >> 3) * lda + 2 * lc;
    const int64_t boff = (int64_t)(lane >> 3) * ldb + 2 * lc;
    // fragment reads: row (tile base) + l % 16, k = 4 m + l / 16 -> logical chunk 2 m + l / 32,
    // double (l / 16) % 2; h = (l % 16) / 2 for every 16-row tile
    uint32_t fo[4];
    const int fr = lane & 15;
#pragma unroll
    for (int m = 0; m < 4; ++m)
        fo[m] = (uint32_t)(fr * 128 + 16 * ((2 * m + (lane >> 5)) ^ (fr >> 1)) + 8 * ((lane >> 4) & 1));
    const uint32_t abyte = (uint32_t)(wa * 64 * 128), bbyte = (uint32_t)((DM + wb * 64) * 128);
    g64_issue(smem, abase(0), lda, bbase(0), ldb, aoff, boff, wave);
    char* cur = smem;
    char* nxt = smem + kDStage;
    for (int k0 = 0; k0 < nk; k0 += DKS) {
        __builtin_amdgcn_s_waitcnt(0xF70);                 // vmcnt(0): this wave's part of slice k0 is in LDS
        __syncthreads();                                   // all of it; the other stage no longer read
        const bool more = k0 + DKS < nk;
        const int kn = more ? k0 + DKS : k0;
        g64_step(acc, cur, nxt, more, abase(kn), lda, bbase(kn), ldb, aoff, boff, wave, fo, abyte, bbyte);
        char* t = cur;
        cur = nxt;
        nxt = t;
    }
}

__device__ inline bool g64_active(const Gemm64Args& a, int r) {
    return a.gate ? a.gate[(int64_t)r * a.gate_stride] != 0 : true;
}

__global__ __launch_bounds__(kThreads) void k_gemm64_pack(Gemm64Args a) {
    const int r = blockIdx.y;
    if (!g64_active(a, r)) return;
    const int64_t n = (int64_t)a.n1 * a.n2;
    const double beta = a.cg[r].beta;
    const double* Xo = a.Pold + (int64_t)r * n;
    const double* R = a.R + (int64_t)r * n;
    double* P = a.P + (int64_t)r * n;
    typedef double d2 __attribute__((ext_vector_type(2)));
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n / 2; i += (int64_t)gridDim.x * kThreads) {
        const d2 x = ((const d2*)Xo)[i], rr = ((const d2*)R)[i];
        ((d2*)P)[i] = d2{pnew_of(rr[0], x[0], beta), pnew_of(rr[1], x[1], beta)};
    }
}

// The epilogue of a final pass for 4 accumulator values (elements at g + o[v] of the packed
// vectors, d at e + o[v]): y = acc + (sigma2 + d) x, then p.q (CG) or the residual b - y and its
// square (RESID); stores y.  Returns the updated dot-product chain.
__device__ __attribute__((always_inline)) inline double g64_epilogue4(const Gemm64Args& a, doublex4 acc,
                                                                     int64_t g, int64_t e, const int64_t (&o)[4],
                                                                     double dot) {
    const int epi = a.epi;
    double xv[4], bv[4], dv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        xv[v] = epi != EPI_STORE ? a.Ep[g + o[v]] : 0.0;
        bv[v] = (epi == EPI_RESID || epi == EPI_RESID_CG) ? a.Er[g + o[v]] : 0.0;
        dv[v] = a.dvec ? a.dvec[e + o[v]] : 0.0;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        double y = acc[v];
        if (epi != EPI_STORE) y = __builtin_fma(a.sigma2 + dv[v], xv[v], y);
        if (epi == EPI_CG) {
            dot = __builtin_fma(xv[v], y, dot);
        } else if (epi == EPI_RESID || epi == EPI_RESID_CG) {
            y = bv[v] - y;
            dot = __builtin_fma(y, y, dot);
        }
        a.Y[g + o[v]] = y;
    }
    return dot;
}

// Per right-hand side reduction of the final pass's dot products and its consequence: the CG
// step length (or a breakdown), the true residual of a reliable update, or a refinement sweep's
// verdict.  tpr blocks per right-hand side, this block being number t of right-hand side r.
__device__ inline void g64_finish(const Gemm64Args& a, int r, int tpr, int t, double dot, double* red) {
    const int epi = a.epi;
    if (epi != EPI_CG && epi != EPI_RESID && epi != EPI_RESID_CG) return;
    const double s = block_sum8(dot, red);
    double tot;
    if (last_block_reduce8(s, a.partials + (int64_t)r * a.part_stride, a.counters + r, tpr, t, &tot, red) &&
        threadIdx.x == 0) {
        if (epi == EPI_CG) {
            CgState& st = a.cg[r];
            if (!(tot > 0.0) || !finite_d(tot)) {
                st.status = finite_d(tot) ? COLA_ERR_NOT_SPD : COLA_ERR_NONFINITE;
                st.active = 0;
                atomicSub(&a.cnt->num_active, 1);
            } else {
                st.alpha = st.rho / tot;
            }
        } else if (epi == EPI_RESID_CG) {
            a.cg[r].rho_true = tot;
        } else {
            outer_residual(a.outer[r], tot, a.cnt);
        }
    }
}

// G1: A = rows of [V_1; ..; V_J] (256 per tile, one term), B = rows of X (128 per tile, one
// right-hand side); the accumulator tile is T_r[b][(j, a')] with a' along the lanes.  The
// mode passes of a one-term three-mode operator are this kernel with J = 1, n1 = the rows per
// right-hand side and n2 = the contracted (and output) mode: T is then Out[r][b][a'], the output
// stored new mode first.  FINAL (three-mode, J = 1): the last pass, whose Out is the product in
// its own layout, with the epilogue of the final pass instead of a plain store.
template <bool FINAL>
__global__ __launch_bounds__(kGT) void k_gemm64_t(Gemm64Args a) {
    __shared__ __attribute__((aligned(16))) char smem[2 * kDStage];
    __shared__ double red[8];
    const int Mt = a.J * a.n2 / DM, Nt = a.nrhs * a.n1 / DN;
    const int L = xcd_linear(blockIdx.x, Mt * Nt);
    const int mt = L % Mt, nt = L / Mt;                    // the A panels of all terms cycle fastest
    const int64_t m0 = (int64_t)mt * DM, n0 = (int64_t)nt * DN;
    const int r = (int)(n0 / a.n1);
    if (!g64_active(a, r)) return;
    const int64_t n2 = a.n2;
    const double* Ab = a.V + m0 * n2;                      // rows (j, b) of the stacked factors
    const double* Bb = a.X + n0 * n2;                      // rows (r, a') of X
    doublex4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
    gemm64_tile(acc, a.n2, [&](int k0) { return Ab + k0; }, n2, [&](int k0) { return Bb + k0; }, n2, smem);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, wa = wave >> 1, wb = wave & 1;
    const int64_t ldt = (int64_t)a.J * a.n1;
    const int jt = (int)(m0 / n2);
    const int64_t b_lane = m0 - (int64_t)jt * n2 + wa * 64 + (lane >> 4);
    const int64_t a_lane = n0 - (int64_t)r * a.n1 + wb * 64 + (lane & 15);
    if constexpr (!FINAL) {
        double* const out = a.T + ((int64_t)r * n2 + b_lane) * ldt + (int64_t)jt * a.n1 + a_lane;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) out[(int64_t)(16 * i + 4 * v) * ldt + 16 * j] = acc[i][j][v];
    } else {
        const int64_t n = n2 * a.n1;                       // elements per right-hand side
        const int64_t e_lane = b_lane * a.n1 + a_lane;
        const int64_t g_lane = (int64_t)r * n + e_lane;
        double dot = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                int64_t o[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) o[v] = (int64_t)(16 * i + 4 * v) * a.n1 + 16 * j;
                dot = g64_epilogue4(a, acc[i][j], g_lane, e_lane, o, dot);
            }
        const int bpr = a.n1 / DN;                         // B tiles per right-hand side
        g64_finish(a, r, Mt * bpr, mt + Mt * (nt - r * bpr), dot, red);
    }
}

// G2: A = rows a of [U_1 .. U_J] (k = (j, a')), B = rows b of T_r; the accumulator tile is
// y_r[a][b] with b along the lanes, followed by the epilogue.
__global__ __launch_bounds__(kGT) void k_gemm64_y(Gemm64Args a) {
    __shared__ __attribute__((aligned(16))) char smem[2 * kDStage];
    __shared__ double red[8];
    const int tn = a.n2 / DN, tpr = (a.n1 / DM) * tn;
    const int L = xcd_linear(blockIdx.x, a.nrhs * tpr);
    const int r = L / tpr, t = L % tpr;
    if (!g64_active(a, r)) return;
    const int a0 = (t / tn) * DM, b0 = (t % tn) * DN;
    const int64_t n1 = a.n1, n2 = a.n2, ldt = (int64_t)a.J * a.n1;
    const double* Tr = a.T + ((int64_t)r * n2 + b0) * ldt;
    doublex4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};
    gemm64_tile(acc, (int)ldt,
                [&](int k0) {
                    const int64_t j = k0 / n1;             // a 16-wide k slice never spans two terms
                    return a.U + j * n1 * n1 + a0 * n1 + (k0 - j * n1);
                },
                n1, [&](int k0) { return Tr + k0; }, ldt, smem);

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, wa = wave >> 1, wb = wave & 1;
    const int64_t n = n1 * n2;
    const int64_t e_lane = (int64_t)(a0 + wa * 64 + (lane >> 4)) * n2 + b0 + wb * 64 + (lane & 15);
    const int64_t g_lane = (int64_t)r * n + e_lane;
    double dot = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            int64_t o[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) o[v] = (int64_t)(16 * i + 4 * v) * n2 + 16 * j;
            dot = g64_epilogue4(a, acc[i][j], g_lane, e_lane, o, dot);
        }
    g64_finish(a, r, tpr, t, dot, red);
}

}  // namespace

bool gemm2_supported(int prec, int Fv, const int64_t* dims) {
    return prec == COLA_PREC_BF16 && Fv == 2 && dims[0] >= BM && dims[1] >= BN && dims[0] % BM == 0 &&
           dims[1] % BN == 0;
}

int64_t gemm2_blocks_per_rhs(int64_t n1, int64_t n2) { return (n1 / BM) * (n2 / BN); }

bool gemm64_supported(int Fv, const int64_t* dims) {
    return Fv == 2 && dims[0] >= DM && dims[1] >= DM && dims[0] % DM == 0 && dims[1] % DM == 0;
}

int64_t gemm64_blocks_per_rhs(int64_t n1, int64_t n2) { return (n1 / DM) * (n2 / DN); }

bool gemm64_3_supported(int Fv, int J, const int64_t* dims) {
    return Fv == 3 && J == 1 && dims[0] >= DM && dims[1] >= DM && dims[2] >= DM && dims[0] % DM == 0 &&
           dims[1] % DM == 0 && dims[2] % DM == 0;
}

int64_t gemm64_3_blocks_per_rhs(int64_t n1, int64_t n2, int64_t n3) { return (n1 / DM) * (n2 * n3 / DN); }

hipError_t launch_gemm64_pass(const Gemm64Args& a, bool final, hipStream_t s) {
    if (a.n2 % DM || a.n1 % DN || a.n1 < DN || a.n2 < DM || a.nrhs < 1 || a.J != 1 || !a.X || !a.V)
        return hipErrorInvalidValue;
    if (final) {
        const bool cg = a.epi == EPI_CG;
        const bool resid = a.epi == EPI_RESID || a.epi == EPI_RESID_CG;
        if ((cg && !a.cg) || (resid && !a.Er) || (a.epi == EPI_RESID && !a.outer) ||
            (a.epi == EPI_RESID_CG && !a.cg) || (a.epi != EPI_STORE && !a.Ep) || !a.Y)
            return hipErrorInvalidValue;
    } else if (!a.T) {
        return hipErrorInvalidValue;
    }
    const int64_t T = (int64_t)(a.n2 / DM) * (a.nrhs * (int64_t)a.n1 / DN);
    if (final) hipLaunchKernelGGL(k_gemm64_t<true>, dim3((unsigned)T), dim3(kGT), 0, s, a);
    else hipLaunchKernelGGL(k_gemm64_t<false>, dim3((unsigned)T), dim3(kGT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gemm64(const Gemm64Args& a, int stage, hipStream_t s) {
    const int64_t dims[2] = {a.n1, a.n2};
    if (!gemm64_supported(2, dims) || a.nrhs < 1 || a.J < 1) return hipErrorInvalidValue;
    const bool cg = a.epi == EPI_CG;
    const bool resid = a.epi == EPI_RESID || a.epi == EPI_RESID_CG;
    if ((cg && (!a.R || !a.P || !a.Pold || !a.cg)) || (resid && !a.Er) || (a.epi == EPI_RESID && !a.outer) ||
        (a.epi == EPI_RESID_CG && !a.cg) || (a.epi != EPI_STORE && !a.Ep))
        return hipErrorInvalidValue;
    if (stage == 0) {
        if (!cg) return hipSuccess;
        const int64_t n2h = (int64_t)a.n1 * a.n2 / 2;
        const int64_t bx = std::min<int64_t>(512, (n2h + kThreads - 1) / kThreads);
        hipLaunchKernelGGL(k_gemm64_pack, dim3((unsigned)bx, (unsigned)a.nrhs), dim3(kThreads), 0, s, a);
    } else if (stage == 1) {
        const int64_t T = (int64_t)(a.J * a.n2 / DM) * (a.nrhs * (int64_t)a.n1 / DN);
        hipLaunchKernelGGL(k_gemm64_t<false>, dim3((unsigned)T), dim3(kGT), 0, s, a);
    } else {
        const int64_t T = (int64_t)a.nrhs * gemm64_blocks_per_rhs(a.n1, a.n2);
        hipLaunchKernelGGL(k_gemm64_y, dim3((unsigned)T), dim3(kGT), 0, s, a);
    }
    return hipGetLastError();
}

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
