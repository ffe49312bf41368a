// Mode contraction pass of the Kronecker MVM on gfx950 matrix cores.
//
// A Kronecker term applied to x (row-major vec) multiplies every tensor mode
// of X = x.reshape(n1, .., nF) by its factor; the MVM cost of Table 2
// (tau_A N_B + N_A tau_B) is exactly the sum of these per-mode products.
// Each pass here is one such mode product, written as a batched GEMM with a
// small inner dimension (the mode size) and staged through LDS:
//
//   ROWS  (last mode):  Y[g, i]    = sum_l X[g, l] K[i, l]     (g: all leading indices)
//   COLS  (other modes): Y[g, i, b] = sum_l K[i, l] X[g, l, b]  (b: trailing indices)
//
// Operands are staged in LDS as [row][k] tiles (k contiguous) and fed to
// 16x16 MFMA tiles; each of the 4 waves owns a (16*WM) x (16*WN) sub-tile.
// Precision policies: FP64 (v_mfma_f64_16x16x4f64), FP32 (v_mfma_f32_16x16x4f32),
// BF16 (v_mfma_f32_16x16x32_bf16, FP32 accumulation) and BF16x3 (each operand
// split into three bf16 parts; the six leading cross products are summed).
//
// The last pass of an MVM carries the fused epilogues of the CG iteration
// (the diagonal term of the Sum, the search-direction update and the partial
// dot product p.Ap) or of the FP64 refinement residual r = b - A x.
#include "contract.h"

namespace cola {

// ----------------------------------------------------------------------------
// precision policies
struct PolF64 {
    using V = double; using Fac = double; using L = double; using Acc = doublex4;
    static constexpr int KT = 16, KSTEP = 4, NS = 1, KP = KT + 2;
};
struct PolF32 {
    using V = float; using Fac = float; using L = float; using Acc = floatx4;
    static constexpr int KT = 32, KSTEP = 4, NS = 1, KP = KT + 4;
};
struct PolBF16 {
    using V = float; using Fac = __bf16; using L = __bf16; using Acc = floatx4;
    static constexpr int KT = 32, KSTEP = 32, NS = 1, KP = KT + 8;
};
struct PolBF16X3 {
    using V = float; using Fac = __bf16; using L = __bf16; using Acc = floatx4;
    static constexpr int KT = 32, KSTEP = 32, NS = 3, KP = KT + 8;
};

template <class P> struct IsBf { static constexpr bool value = false; };
template <> struct IsBf<PolBF16> { static constexpr bool value = true; };
template <> struct IsBf<PolBF16X3> { static constexpr bool value = true; };

__device__ inline floatx4 mma(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline doublex4 mma(double a, double b, doublex4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline floatx4 mma(bf16x8 a, bf16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Split a working-precision value into the policy's LDS parts.
template <class P>
__device__ inline void split_value(typename P::V v, typename P::L* out) {
    if constexpr (!IsBf<P>::value) {
        out[0] = v;
    } else {
        __bf16 h = (__bf16)v;                  // round to nearest even
        out[0] = h;
        if constexpr (P::NS == 3) {
            float r1 = v - (float)h;
            __bf16 m = (__bf16)r1;
            float r2 = r1 - (float)m;
            out[1] = m;
            out[2] = (__bf16)r2;
        }
    }
}

__device__ inline bool gate_of(const PassArgs& a, int64_t rhs) {
    return a.gate ? a.gate[rhs * a.gate_stride] != 0 : true;
}

// 4 consecutive elements (the address is a multiple of 4 elements).
__device__ inline void load4(const float* p, float* o) {
    const floatx4 v = *(const floatx4*)p;
    o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
}
__device__ inline void load4(const double* p, double* o) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 a = *(const d2*)p, b = *(const d2*)(p + 2);
    o[0] = a[0]; o[1] = a[1]; o[2] = b[0]; o[3] = b[1];
}
__device__ inline void load4(const __bf16* p, __bf16* o) {
    typedef __bf16 b4 __attribute__((ext_vector_type(4)));
    const b4 v = *(const b4*)p;
    o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
}
__device__ inline void store4(float* p, const float* v) { *(floatx4*)p = floatx4{v[0], v[1], v[2], v[3]}; }
__device__ inline void store4(double* p, const double* v) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    *(d2*)p = d2{v[0], v[1]};
    *(d2*)(p + 2) = d2{v[2], v[3]};
}

template <class P, int WM, int WN, bool ROWS>
__global__ __launch_bounds__(kThreads) void k_contract(PassArgs a) {
    using V = typename P::V; using Fac = typename P::Fac; using L = typename P::L;
    using Acc = typename P::Acc;
    constexpr int MT = 32 * WM, NT = 32 * WN, KT = P::KT, KP = P::KP, NS = P::NS;
    constexpr int EPAD = sizeof(V) == 8 ? 2 : 4;
    constexpr int EW = 16 * WN + EPAD;                       // epilogue row stride (elements)
    // COLS, FP32/FP64: the vector tile is staged as [k][n] (as it lies in
    // memory) with a row pitch of 16 (mod 64) banks, which keeps both the
    // 16-byte staging writes and the MFMA operand reads free of bank
    // conflicts; the bf16 policies keep [n][k] for their 8-wide k operands.
    constexpr bool BKN = !ROWS && !IsBf<P>::value;
    constexpr int NTP = NT + (sizeof(L) == 8 ? 8 : 16);
    constexpr size_t B_ELEMS = BKN ? (size_t)KT * NTP : (size_t)NT * KP;
    constexpr size_t AB_BYTES = sizeof(L) * NS * ((size_t)MT * KP + B_ELEMS);
    constexpr size_t E_BYTES = sizeof(V) * 4 * 16 * (size_t)EW;
    constexpr size_t SMEM = AB_BYTES > E_BYTES ? AB_BYTES : E_BYTES;
    __shared__ __attribute__((aligned(16))) char smem[SMEM];
    __shared__ double red[4];
    L* As = (L*)smem;                      // [NS][MT][KP]
    L* Bs = As + NS * MT * KP;             // [NS][NT][KP], or [KT][NTP] when BKN

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int nk = a.nk;
    const int64_t k_plane = a.k_plane;
    const bool kvec = (nk % 4) == 0;                       // factor rows / ROWS vectors load 4-wide
    const bool bvec = (a.B % 4) == 0;                      // COLS vectors load 4-wide

    int64_t g = 0, m0, n0, nBt = 1;
    int nMt = 1, tout;
    if constexpr (ROWS) {
        const int nNt = (nk + NT - 1) / NT;
        m0 = (int64_t)blockIdx.x * MT;
        n0 = (int64_t)(blockIdx.y % nNt) * NT;
        tout = blockIdx.y / nNt;
        if (a.gate) {
            const int64_t last = (m0 + MT < a.G ? m0 + MT : a.G) - 1;
            bool any = false;
            for (int64_t r = m0 / a.a_per_rhs; r <= last / a.a_per_rhs; ++r) any |= gate_of(a, r);
            if (!any) return;
        }
    } else {
        nBt = (a.B + NT - 1) / NT;
        g = blockIdx.x / nBt;
        n0 = (int64_t)(blockIdx.x % nBt) * NT;
        nMt = (nk + MT - 1) / MT;
        m0 = (int64_t)(blockIdx.y % nMt) * MT;
        tout = blockIdx.y / nMt;
        if (!gate_of(a, g / a.a_per_rhs)) return;
    }

    Acc acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = Acc{0, 0, 0, 0};

    double beta_blk = 0.0;
    if (!ROWS && a.pnew) beta_blk = a.cg[g / a.a_per_rhs].beta;
    // every element of this block's output tile exists and rows are 16-byte aligned
    const bool tile_full = !ROWS && bvec && (m0 + MT <= nk) && (n0 + NT <= a.B);

    // stage a k-contiguous [rows][KT] tile of a factor (4 elements per step)
    auto stage_factor = [&](L* dst, const Fac* Kp, int64_t r0, int rows, int k0) {
        for (int e = tid; e < rows * (KT / 4); e += kThreads) {
            const int m = e / (KT / 4), k = (e % (KT / 4)) * 4;
            const int64_t gm = r0 + m;
            const int gk = k0 + k;
#pragma unroll
            for (int sp = 0; sp < NS; ++sp) {
                Fac f[4] = {(Fac)0.0f, (Fac)0.0f, (Fac)0.0f, (Fac)0.0f};
                if (gm < nk) {
                    const Fac* src = Kp + sp * k_plane + gm * nk + gk;
                    if (kvec && gk + 3 < nk) {
                        load4(src, f);
                    } else {
#pragma unroll
                        for (int c = 0; c < 4; ++c) if (gk + c < nk) f[c] = src[c];
                    }
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) dst[(sp * rows + m) * KP + k + c] = (L)f[c];
            }
        }
    };

    // The CG epilogue's streaming operands (r and p_old) do not depend on the
    // contraction: issue their loads now so they arrive while the MFMA loop runs.
    constexpr bool PREF = false;   // measured slower: the extra registers cost more occupancy than the early loads gained
    constexpr int CHN = (16 * WN) / 4;                       // 4-column chunks per staged row
    V pre_r[PREF ? WM : 1][PREF ? WN : 1][4], pre_p[PREF ? WM : 1][PREF ? WN : 1][4];
    const bool use_pref = PREF && a.epi == EPI_CG && bvec;
    if constexpr (PREF) {
        if (use_pref) {
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int c = 0; c < WN; ++c) {
                    const int t2 = lane + 64 * c;
                    const int r = t2 / CHN, c4 = (t2 % CHN) * 4;
                    const int64_t m = m0 + wm * WM * 16 + i * 16 + r;
                    const int64_t n = n0 + wn * WN * 16 + c4;
                    if (m < nk && n + 3 < a.B) {
                        const int64_t idx = g * (int64_t)nk * a.B + m * a.B + n;
                        load4((const V*)a.Er + idx, pre_r[i][c]);
                        load4((const V*)a.Ep + idx, pre_p[i][c]);
                    }
                }
        }
    }

    for (int t = 0; t < a.nsum; ++t) {
        const int tt = (a.nsum > 1) ? t : tout;
        const Fac* Kp = (const Fac*)a.K + (int64_t)tt * a.k_tstride;
        const V* Xp = (const V*)a.X + (int64_t)tt * a.x_tstride;
        const V* Rp = (const V*)a.R + (int64_t)tt * a.x_tstride;
        for (int k0 = 0; k0 < nk; k0 += KT) {
            if constexpr (ROWS) {
                // A: vector rows X[g, k] (k contiguous), B: factor rows K[i, k]
                for (int e = tid; e < MT * (KT / 4); e += kThreads) {
                    const int m = e / (KT / 4), k = (e % (KT / 4)) * 4;
                    const int64_t gm = m0 + m;
                    const int gk = k0 + k;
                    V v[4] = {0, 0, 0, 0};
                    if (gm < a.G) {
                        const int64_t idx = gm * nk + gk;
                        if (kvec && gk + 3 < nk) {
                            load4(Xp + idx, v);
                            if (a.pnew) {
                                V rr[4];
                                load4(Rp + idx, rr);
                                const double be = a.cg[gm / a.a_per_rhs].beta;
#pragma unroll
                                for (int c = 0; c < 4; ++c) v[c] = pnew_of(rr[c], v[c], be);
                            }
                        } else {
#pragma unroll
                            for (int c = 0; c < 4; ++c)
                                if (gk + c < nk) {
                                    v[c] = Xp[idx + c];
                                    if (a.pnew) v[c] = pnew_of(Rp[idx + c], v[c], a.cg[gm / a.a_per_rhs].beta);
                                }
                        }
                    }
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        L parts[NS];
                        split_value<P>(v[c], parts);
#pragma unroll
                        for (int sp = 0; sp < NS; ++sp) As[(sp * MT + m) * KP + k + c] = parts[sp];
                    }
                }
                stage_factor(Bs, Kp, n0, NT, k0);
            } else {
                // A: factor rows K[i, k], B: vector X[g, k, b] (b contiguous) stored as [b][k]
                stage_factor(As, Kp, m0, MT, k0);
                if (BKN && tile_full && k0 + KT <= nk) {
                    // whole tile in range: straight-line 16-byte loads, all issued before use
                    constexpr int NE = (KT * (NT / 4) + kThreads - 1) / kThreads;
                    V v[NE][4], rr4[NE][4];
#pragma unroll
                    for (int q = 0; q < NE; ++q) {
                        const int e = tid + kThreads * q;
                        if (e < KT * (NT / 4)) {
                            const int k = e / (NT / 4), n = (e % (NT / 4)) * 4;
                            const int64_t idx = (g * nk + k0 + k) * a.B + n0 + n;
                            load4(Xp + idx, v[q]);
                            if (a.pnew) load4(Rp + idx, rr4[q]);
                        }
                    }
#pragma unroll
                    for (int q = 0; q < NE; ++q) {
                        const int e = tid + kThreads * q;
                        if (e < KT * (NT / 4)) {
                            const int k = e / (NT / 4), n = (e % (NT / 4)) * 4;
#pragma unroll
                            for (int c = 0; c < 4; ++c)
                                Bs[k * NTP + n + c] = (L)(a.pnew ? pnew_of(rr4[q][c], v[q][c], beta_blk) : v[q][c]);
                        }
                    }
                } else
                for (int e = tid; e < KT * (NT / 4); e += kThreads) {
                    const int k = e / (NT / 4), n = (e % (NT / 4)) * 4;
                    const int gk = k0 + k;
                    const int64_t gn = n0 + n;
                    V v[4] = {0, 0, 0, 0};
                    if (gk < nk) {
                        const int64_t idx = (g * nk + gk) * a.B + gn;
                        if (bvec && gn + 3 < a.B) {
                            load4(Xp + idx, v);
                            if (a.pnew) {
                                V rr[4];
                                load4(Rp + idx, rr);
#pragma unroll
                                for (int c = 0; c < 4; ++c) v[c] = pnew_of(rr[c], v[c], beta_blk);
                            }
                        } else {
#pragma unroll
                            for (int c = 0; c < 4; ++c)
                                if (gn + c < a.B) {
                                    v[c] = Xp[idx + c];
                                    if (a.pnew) v[c] = pnew_of(Rp[idx + c], v[c], beta_blk);
                                }
                        }
                    }
                    if constexpr (BKN) {
#pragma unroll
                        for (int c = 0; c < 4; ++c) Bs[k * NTP + n + c] = (L)v[c];
                    } else {
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            L parts[NS];
                            split_value<P>(v[c], parts);
#pragma unroll
                            for (int sp = 0; sp < NS; ++sp) Bs[(sp * NT + n + c) * KP + k] = parts[sp];
                        }
                    }
                }
            }
            __syncthreads();
            // ---- MFMA over the staged K slice ----
#pragma unroll
            for (int kk = 0; kk < KT; kk += P::KSTEP) {
                if constexpr (!IsBf<P>::value) {
                    L av[WM], bv[WN];
#pragma unroll
                    for (int i = 0; i < WM; ++i)
                        av[i] = As[(wm * WM * 16 + i * 16 + (lane & 15)) * KP + kk + (lane >> 4)];
#pragma unroll
                    for (int j = 0; j < WN; ++j) {
                        if constexpr (BKN) bv[j] = Bs[(kk + (lane >> 4)) * NTP + wn * WN * 16 + j * 16 + (lane & 15)];
                        else bv[j] = Bs[(wn * WN * 16 + j * 16 + (lane & 15)) * KP + kk + (lane >> 4)];
                    }
#pragma unroll
                    for (int i = 0; i < WM; ++i)
#pragma unroll
                        for (int j = 0; j < WN; ++j) acc[i][j] = mma(av[i], bv[j], acc[i][j]);
                } else {
                    bf16x8 av[NS][WM], bv[NS][WN];
#pragma unroll
                    for (int sp = 0; sp < NS; ++sp) {
#pragma unroll
                        for (int i = 0; i < WM; ++i)
                            av[sp][i] = *(const bf16x8*)&As[(sp * MT + wm * WM * 16 + i * 16 + (lane & 15)) * KP + kk +
                                                           8 * (lane >> 4)];
#pragma unroll
                        for (int j = 0; j < WN; ++j)
                            bv[sp][j] = *(const bf16x8*)&Bs[(sp * NT + wn * WN * 16 + j * 16 + (lane & 15)) * KP + kk +
                                                           8 * (lane >> 4)];
                    }
#pragma unroll
                    for (int i = 0; i < WM; ++i)
#pragma unroll
                        for (int j = 0; j < WN; ++j) {
                            if constexpr (NS == 1) {
                                acc[i][j] = mma(av[0][i], bv[0][j], acc[i][j]);
                            } else {
                                // smallest products first: lo*hi, hi*lo, mid*mid, mid*hi, hi*mid, hi*hi
                                acc[i][j] = mma(av[2][i], bv[0][j], acc[i][j]);
                                acc[i][j] = mma(av[0][i], bv[2][j], acc[i][j]);
                                acc[i][j] = mma(av[1][i], bv[1][j], acc[i][j]);
                                acc[i][j] = mma(av[1][i], bv[0][j], acc[i][j]);
                                acc[i][j] = mma(av[0][i], bv[1][j], acc[i][j]);
                                acc[i][j] = mma(av[0][i], bv[0][j], acc[i][j]);
                            }
                        }
                }
            }
            __syncthreads();
        }
    }

    // ---- epilogue: each wave stages one 16-row slice of its sub-tile in LDS
    // and then walks it 4 columns at a time, so global accesses are 16-byte
    // vectors along the contiguous dimension ----
    double dot = 0.0;
    V* Y = (V*)a.Y + (int64_t)tout * a.y_tstride;
    double beta_e = 0.0;
    if (!ROWS && a.epi == EPI_CG) beta_e = a.cg[g].beta;
    V* Ew = (V*)smem + wave * 16 * EW;
    constexpr int CH = (16 * WN) / 4;                        // 4-column chunks per staged row
#pragma unroll
    for (int i = 0; i < WM; ++i) {
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                Ew[acc_row(acc[i][j][v], lane, v) * EW + j * 16 + (lane & 15)] = (V)acc[i][j][v];
        __syncthreads();
        if (tile_full) {
            // uniform fast path: every chunk is a full 16-byte vector; all loads first
            V u4[WN][4], w4v[WN][4], d4v[WN][4];
            const bool need_p = a.epi != EPI_STORE, need_r = a.epi == EPI_CG || a.epi == EPI_RESID ||
                                                             a.epi == EPI_RESID_CG;
#pragma unroll
            for (int cc = 0; cc < WN; ++cc) {
                const int t2 = lane + 64 * cc;
                const int r = t2 / CH, c4 = (t2 % CH) * 4;
                const int64_t m = m0 + wm * WM * 16 + i * 16 + r;
                const int64_t e0 = m * a.B + n0 + wn * WN * 16 + c4;
                const int64_t idx = g * (int64_t)nk * a.B + e0;
                if (need_p) load4((const V*)a.Ep + idx, u4[cc]);
                if (need_r) load4((const V*)a.Er + idx, w4v[cc]);
                if (need_p && a.dvec) load4((const V*)a.dvec + e0, d4v[cc]);
            }
#pragma unroll
            for (int cc = 0; cc < WN; ++cc) {
                const int t2 = lane + 64 * cc;
                const int r = t2 / CH, c4 = (t2 % CH) * 4;
                const int64_t m = m0 + wm * WM * 16 + i * 16 + r;
                const int64_t e0 = m * a.B + n0 + wn * WN * 16 + c4;
                const int64_t idx = g * (int64_t)nk * a.B + e0;
                V val[4], out[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) val[c] = Ew[r * EW + c4 + c];
                if (a.epi == EPI_STORE) {
                    store4(Y + idx, val);
                    continue;
                }
                V dg[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) dg[c] = (V)a.sigma2 + (a.dvec ? d4v[cc][c] : (V)0);
                if (a.epi == EPI_CG) {
                    V pn[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        pn[c] = pnew_of(w4v[cc][c], u4[cc][c], beta_e);
                        out[c] = val[c] + dg[c] * pn[c];
                        dot += (double)pn[c] * (double)out[c];
                    }
                    store4(Y + idx, out);
                    store4((V*)a.Epout + idx, pn);
                } else if (a.epi == EPI_MATVEC) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) out[c] = val[c] + dg[c] * u4[cc][c];
                    store4(Y + idx, out);
                } else {
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        out[c] = w4v[cc][c] - (val[c] + dg[c] * u4[cc][c]);
                        dot += (double)out[c] * (double)out[c];
                    }
                    store4(Y + idx, out);
                }
            }
            __syncthreads();
            continue;
        }
#pragma unroll
        for (int cc = 0; cc < WN; ++cc) {               // 16 * CH = 64 * WN chunks: WN per lane
            const int t2 = lane + 64 * cc;
            const int r = t2 / CH, c4 = (t2 % CH) * 4;
            const int64_t m = m0 + wm * WM * 16 + i * 16 + r;
            const int64_t n = n0 + wn * WN * 16 + c4;
            V val[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) val[c] = Ew[r * EW + c4 + c];
            if constexpr (ROWS) {
                if (m < a.G) {
                    V* dst = Y + m * nk + n;
                    if (kvec && n + 3 < nk) store4(dst, val);
                    else
                        for (int c = 0; c < 4; ++c) if (n + c < nk) dst[c] = val[c];
                }
            } else if (m < nk) {
                const int64_t e0 = m * a.B + n;
                const int64_t idx = g * (int64_t)nk * a.B + e0;
                const bool full = bvec && n + 3 < a.B;
                const int cnt = full ? 4 : (int)((a.B - n) < 4 ? (a.B - n > 0 ? a.B - n : 0) : 4);
                V out[4] = {val[0], val[1], val[2], val[3]};
                if (a.epi == EPI_STORE) {
                    if (full) store4(Y + idx, out);
                    else for (int c = 0; c < cnt; ++c) Y[idx + c] = out[c];
                } else {
                    V dg[4], u[4], w4[4];
                    for (int c = 0; c < 4; ++c) dg[c] = (V)a.sigma2;
                    if (full) {
                        if (a.dvec) { V d4[4]; load4((const V*)a.dvec + e0, d4); for (int c = 0; c < 4; ++c) dg[c] += d4[c]; }
                        if constexpr (PREF) {
                            if (use_pref) {
#pragma unroll
                                for (int c = 0; c < 4; ++c) { u[c] = pre_p[i][cc][c]; w4[c] = pre_r[i][cc][c]; }
                            } else {
                                load4((const V*)a.Ep + idx, u);
                                if (a.epi != EPI_MATVEC) load4((const V*)a.Er + idx, w4);
                            }
                        } else {
                            load4((const V*)a.Ep + idx, u);
                            if (a.epi != EPI_MATVEC) load4((const V*)a.Er + idx, w4);
                        }
                    } else {
                        for (int c = 0; c < cnt; ++c) {
                            if (a.dvec) dg[c] += ((const V*)a.dvec)[e0 + c];
                            u[c] = ((const V*)a.Ep)[idx + c];
                            if (a.epi != EPI_MATVEC) w4[c] = ((const V*)a.Er)[idx + c];
                        }
                    }
                    if (a.epi == EPI_CG) {
                        V pn[4];
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            pn[c] = pnew_of(w4[c], u[c], beta_e);     // r + beta p_old
                            out[c] = val[c] + dg[c] * pn[c];
                        }
                        for (int c = 0; c < cnt; ++c) dot += (double)pn[c] * (double)out[c];
                        if (full) { store4(Y + idx, out); store4((V*)a.Epout + idx, pn); }
                        else for (int c = 0; c < cnt; ++c) { Y[idx + c] = out[c]; ((V*)a.Epout)[idx + c] = pn[c]; }
                    } else if (a.epi == EPI_RESID || a.epi == EPI_RESID_CG) {
#pragma unroll
                        for (int c = 0; c < 4; ++c) out[c] = w4[c] - (val[c] + dg[c] * u[c]);
                        for (int c = 0; c < cnt; ++c) dot += (double)out[c] * (double)out[c];
                        if (full) store4(Y + idx, out);
                        else for (int c = 0; c < cnt; ++c) Y[idx + c] = out[c];
                    } else {  // EPI_MATVEC
#pragma unroll
                        for (int c = 0; c < 4; ++c) out[c] = val[c] + dg[c] * u[c];
                        if (full) store4(Y + idx, out);
                        else for (int c = 0; c < cnt; ++c) Y[idx + c] = out[c];
                    }
                }
            }
        }
        __syncthreads();
    }

    if constexpr (!ROWS) {
        if (a.epi == EPI_CG || a.epi == EPI_RESID || a.epi == EPI_RESID_CG) {
            const double s = block_sum(dot, red);
            const int64_t nblk = nBt * nMt;
            const int64_t myb = (blockIdx.x % nBt) + nBt * (blockIdx.y % nMt);
            double tot;
            if (last_block_reduce(s, a.partials + g * a.part_stride, a.counters + g, (int)nblk,
                                  (int)myb, &tot, red) && tid == 0) {
                if (a.epi == EPI_CG) {
                    CgState& st = a.cg[g];
                    if (!(tot > 0.0) || !finite_d(tot)) {
                        st.status = finite_d(tot) ? COLA_ERR_NOT_SPD : COLA_ERR_NONFINITE;
                        st.active = 0;
                        atomicSub(&a.cnt->num_active, 1);
                    } else {
                        st.alpha = st.rho / tot;
                    }
                } else if (a.epi == EPI_RESID_CG) {
                    a.cg[g].rho_true = tot;
                } else {
                    outer_residual(a.outer[g], tot, a.cnt);
                }
            }
        }
    }
}

// ----------------------------------------------------------------------------
template <class P, int WM, int WN>
static hipError_t launch_t(bool rows, const PassArgs& a, hipStream_t s) {
    constexpr int MT = 32 * WM, NT = 32 * WN;
    dim3 grid;
    if (rows) {
        const int64_t nNt = (a.nk + NT - 1) / NT;
        grid = dim3((unsigned)((a.G + MT - 1) / MT), (unsigned)(nNt * a.nout), 1);
        hipLaunchKernelGGL((k_contract<P, WM, WN, true>), grid, dim3(kThreads), 0, s, a);
    } else {
        const int64_t nBt = (a.B + NT - 1) / NT;
        const int64_t nMt = (a.nk + MT - 1) / MT;
        grid = dim3((unsigned)(a.G * nBt), (unsigned)(nMt * a.nout), 1);
        hipLaunchKernelGGL((k_contract<P, WM, WN, false>), grid, dim3(kThreads), 0, s, a);
    }
    return hipGetLastError();
}

template <class P>
static hipError_t launch_p(bool rows, const PassArgs& a, TileCfg c, hipStream_t s) {
    switch (c.wm * 8 + c.wn) {
        case 9:  return launch_t<P, 1, 1>(rows, a, s);
        case 10: return launch_t<P, 1, 2>(rows, a, s);
        case 12: return launch_t<P, 1, 4>(rows, a, s);
        case 17: return launch_t<P, 2, 1>(rows, a, s);
        case 18: return launch_t<P, 2, 2>(rows, a, s);
        case 20: return launch_t<P, 2, 4>(rows, a, s);
        case 33: return launch_t<P, 4, 1>(rows, a, s);
        case 34: return launch_t<P, 4, 2>(rows, a, s);
        case 36: return launch_t<P, 4, 4>(rows, a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_contract(int prec, bool rows, const PassArgs& a, TileCfg cfg, hipStream_t s) {
    switch (prec) {
        case COLA_PREC_FP64:   return launch_p<PolF64>(rows, a, cfg, s);
        case COLA_PREC_FP32:   return launch_p<PolF32>(rows, a, cfg, s);
        case COLA_PREC_BF16:   return launch_p<PolBF16>(rows, a, cfg, s);
        case COLA_PREC_BF16X3: return launch_p<PolBF16X3>(rows, a, cfg, s);
        default: return hipErrorInvalidValue;
    }
}

int64_t contract_blocks_per_g(int /*prec*/, const PassArgs& a, TileCfg cfg) {
    const int64_t MT = 32 * cfg.wm, NT = 32 * cfg.wn;
    return ((a.B + NT - 1) / NT) * ((a.nk + MT - 1) / MT);
}

}  // namespace cola
