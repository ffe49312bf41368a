// Kronecker MVM of three-mode FP32 operators with 256-wide modes as three dense GEMMs.
//
// q = (K1 (x) K2 (x) K3) p is evaluated one mode at a time, the per-mode cost
// of Table 2.  With 256-wide modes every mode product is a dense GEMM with a
// 256-deep inner dimension, run on the FP32 matrix cores
// (v_mfma_f32_32x32x2f32).  Each pass contracts the contiguous (last) mode of
// its input and writes its output transposed per right-hand side, new mode
// first, so that the next pass again reads its operand k-contiguous and the
// third pass writes q in the original layout.  The first pass forms the CG
// direction p = r + beta p_old while staging its operand (and writes it back);
// the last pass carries the CG epilogue (diagonal term, p.q, step length).
//
// Block tile 256 x 256, k slice 32, 4 waves of 128 x 128 (4 x 4 MFMA tiles);
// two LDS stages, the next slice loaded during the current slice's MFMAs.
#include "gemm3.h"

#include <cstring>
#include <type_traits>

#include "contract.h"

namespace cola {

typedef float floatx16 __attribute__((ext_vector_type(16)));

namespace {

constexpr int BM = 256, BN = 256, KS = 32;
constexpr int KSP = KS + 4;                      // LDS row pitch (floats): conflict-free 16-byte reads
constexpr int kChunks = BM * KS / 4 / kThreads;  // 16-byte chunks of one operand slice per thread
constexpr int kStage = (BM + BN) * KSP;          // floats of one LDS stage (A and B slices)
constexpr int TP = 128 + 4;                      // epilogue staging pitch (floats)

__device__ inline floatx16 mfma32f(float a, float b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Row of accumulator element v of a 32 x 32 MFMA tile held by `lane`; the
// column is lane % 32.
__device__ inline int row32(int lane, int v) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

__device__ inline int xcd_linear(int b, int T) {
    return (T % 8 == 0) ? (b % 8) * (T / 8) + b / 8 : b;
}

// One pass: C[m][n] = sum_k A[m][k] B[n][k] over all right-hand sides, stored
// as Out[r][n][m - r * rows_per_rhs].
struct PassDesc {
    const float* A;        // rows x K, row-major (right-hand sides stacked)
    const float* R;        // PNEW: residual, same layout as A
    float* Pout;           // PNEW: the direction, written back (aliases A)
    const float* B;        // N x K factor, row-major
    float* Out;
    int64_t rows_per_rhs;
    int32_t K, N;
};

template <bool PNEW, int EPI>
__global__ __launch_bounds__(kThreads) void k_gemm3(Gemm3Args a, PassDesc d) {
    __shared__ __attribute__((aligned(16))) float smem[2 * kStage];
    __shared__ double red[4];
    const int64_t rows = (int64_t)a.nrhs * d.rows_per_rhs;
    const int Mt = (int)(rows / BM), Nt = d.N / BN;
    const int L = xcd_linear(blockIdx.x, Mt * Nt);
    const int mt = L / Nt, nt = L % Nt;                    // N tiles of one row band run together
    const int64_t m0 = (int64_t)mt * BM;
    const int r = (int)(m0 / d.rows_per_rhs);
    if (a.gate && !a.gate[(int64_t)r * a.gate_stride]) return;
    const int n0 = nt * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
    const int crow = tid >> 3, ck = (tid & 7) * 4;
    const int64_t K = d.K;
    const float* Ab = d.A + m0 * K;
    const float* Rb = PNEW ? d.R + m0 * K : nullptr;
    float* Pb = PNEW ? d.Pout + m0 * K : nullptr;
    const float* Bb = d.B + (int64_t)n0 * K;
    const double beta = PNEW ? a.cg[r].beta : 0.0;
    // x += alpha p_old of the previous step, deferred from the vector update:
    // this pass reads p_old anyway and is bound by its MFMAs, not its traffic
    float* Xb = nullptr;
    float xalpha = 0.f;
    if constexpr (PNEW) {
        if (a.Xit) {
            if (threadIdx.x == 0) a.cg[r].xdefer = 1;      // every block stores the same value
            if (a.cg[r].xlag) {
                Xb = a.Xit + m0 * K;
                xalpha = (float)a.cg[r].alpha;
            }
        }
    }
    const uint32_t off = (uint32_t)(crow * K + ck);

    floatx16 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = floatx16{};

    floatx4 ra[kChunks], rr[PNEW ? kChunks : 1], rb[kChunks], rx[PNEW ? kChunks : 1];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < kChunks; ++q) {
            const int64_t o = (int64_t)q * 32 * K + off + k0;
            ra[q] = *(const floatx4*)(Ab + o);
            if constexpr (PNEW) {
                rr[q] = *(const floatx4*)(Rb + o);
                if (Xb) rx[q] = *(const floatx4*)(Xb + o);
            }
            rb[q] = *(const floatx4*)(Bb + o);
        }
    };
    // the direction is formed here, once per element (one N tile: n3 = 256),
    // and written back in place of p_old
    auto stage = [&](int buf, int k0) {
        float* As = smem + buf * kStage;
        float* Bs = As + BM * KSP;
#pragma unroll
        for (int q = 0; q < kChunks; ++q) {
            floatx4 v = ra[q];
            if constexpr (PNEW) {
                if (Xb) {
                    floatx4 xv = rx[q];
#pragma unroll
                    for (int c = 0; c < 4; ++c) xv[c] = __builtin_fmaf(xalpha, v[c], xv[c]);
                    *(floatx4*)(Xb + (int64_t)q * 32 * K + off + k0) = xv;
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) v[c] = pnew_of(rr[q][c], v[c], beta);
                *(floatx4*)(Pb + (int64_t)q * 32 * K + off + k0) = v;
            }
            *(floatx4*)&As[(crow + 32 * q) * KSP + ck] = v;
            *(floatx4*)&Bs[(crow + 32 * q) * KSP + ck] = rb[q];
        }
    };
    // lane half h supplies k = kk + 4 h + s at MFMA step s, for A and B alike
    auto compute = [&](int buf) {
        const float* As = smem + buf * kStage;
        const float* Bs = As + BM * KSP;
#pragma unroll
        for (int kk = 0; kk < KS; kk += 8) {
            floatx4 av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                av[i] = *(const floatx4*)&As[(wm * 128 + i * 32 + (lane & 31)) * KSP + kk + 4 * (lane >> 5)];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                bv[j] = *(const floatx4*)&Bs[(wn * 128 + j * 32 + (lane & 31)) * KSP + kk + 4 * (lane >> 5)];
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = mfma32f(av[i][s], bv[j][s], acc[i][j]);
        }
    };

    load(0);
    stage(0, 0);
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < d.K; k0 += KS) {
        const bool more = k0 + KS < d.K;
        load(more ? k0 + KS : k0);                         // unconditional: stays in flight
        __builtin_amdgcn_sched_barrier(0);                 // keep the loads ahead of the MFMAs
        compute(buf);
        if (more) stage(buf ^ 1, k0 + KS);
        __syncthreads();
        buf ^= 1;
    }

    // epilogue: transposed store, one 32-column slice of the wave's sub-tile at
    // a time, staged in LDS as [column][row] so rows leave as 16-byte vectors
    const int64_t mloc = (m0 - (int64_t)r * d.rows_per_rhs) + wm * 128;
    const int64_t rhs_base = (int64_t)r * d.N * d.rows_per_rhs;
    float* Ef = smem + wave * 32 * TP;
    const float s2 = (float)a.sigma2;
    double dacc[4] = {0.0, 0.0, 0.0, 0.0};                 // p.q in FP64, four short chains
    // chunk c of slice jt: column jt*32 + 2c + lane/32, rows (lane % 32)*4 .. +3 of the
    // wave's sub-tile; the lane part of the offset is fixed, the rest uniform
    const int64_t lane_pos = (int64_t)(n0 + wn * 128 + (lane >> 5)) * d.rows_per_rhs + mloc + (lane & 31) * 4;
    auto pos_of = [&](int jt, int c) -> int64_t { return lane_pos + (int64_t)(jt * 32 + 2 * c) * d.rows_per_rhs; };
    // the direction (or x) of a slice is loaded before the slice is staged, so
    // its latency overlaps the staging and the barrier
    floatx4 pv[EPI == EPI_STORE ? 1 : 16];
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) {
        __builtin_amdgcn_sched_barrier(0);                 // one slice's loads in flight at a time
        if constexpr (EPI != EPI_STORE) {
#pragma unroll
            for (int c = 0; c < 16; ++c) pv[c] = *(const floatx4*)(a.X + rhs_base + pos_of(jt, c));
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int v = 0; v < 16; ++v) Ef[(lane & 31) * TP + i * 32 + row32(lane, v)] = acc[i][jt][v];
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const int id = lane + 64 * c;
            const int col = id >> 5, m4 = (id & 31) * 4;
            const int64_t pos = pos_of(jt, c);
            const floatx4 y = *(const floatx4*)&Ef[col * TP + m4];
            if constexpr (EPI == EPI_STORE) {
                *(floatx4*)(d.Out + rhs_base + pos) = y;
            } else {
                const floatx4 p = pv[c];                                       // p_new (CG) or x
                floatx4 dg = floatx4{s2, s2, s2, s2};
                if (a.dvec) dg += *(const floatx4*)(a.dvec + pos);
                floatx4 q;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    q[u] = y[u] + dg[u] * p[u];
                    if constexpr (EPI == EPI_CG) dacc[u] = __builtin_fma((double)p[u], (double)q[u], dacc[u]);
                }
                *(floatx4*)(d.Out + rhs_base + pos) = q;
            }
        }
        __syncthreads();
    }
    if constexpr (EPI == EPI_CG) {
        const double sum = block_sum((dacc[0] + dacc[1]) + (dacc[2] + dacc[3]), red);
        const int tpr = (int)(d.rows_per_rhs / BM) * Nt;
        const int t = (int)((m0 - (int64_t)r * d.rows_per_rhs) / BM) * Nt + nt;
        double tot;
        if (last_block_reduce(sum, a.partials + (int64_t)r * a.part_stride, a.counters + r, tpr, t, &tot, red) &&
            threadIdx.x == 0) {
            CgState& st = a.cg[r];
            st.xlag = 0;                                   // the first pass has caught x up
            if (!(tot > 0.0) || !finite_d(tot)) {
                st.status = finite_d(tot) ? COLA_ERR_NOT_SPD : COLA_ERR_NONFINITE;
                st.active = 0;
                atomicSub(&a.cnt->num_active, 1);
            } else {
                st.alpha = st.rho / tot;
            }
        }
    }
}


// ---------------------------------------------------------------------------
// BF16x3 working precision: the same three passes on the BF16 matrix cores.
// Every FP32 operand v is split into three BF16 parts while it is staged,
// v = h + m + l (each part the round-to-nearest-even BF16 of the remainder),
// the factor (FP32 working copy) the same way.  Each k step
// forms the six leading cross products hh, hm, mh, hl, lh and mm with
// v_mfma_f32_32x32x16_bf16 into one FP32 accumulator; the dropped products
// (ml, lm, ll) are below FP32 rounding, so the pass matches the FP32 engine's
// accuracy at the BF16 rate.
//
// The factor is the MFMA's A operand and the vector its B operand, so the
// accumulator tile is the pass output already transposed: lanes 0..31 of a
// row hold 32 consecutive entries of one output column Out[r][n][.], and the
// epilogue stores straight from the accumulators in full 128-byte lines.
//
// Block tile 256 (factor rows n) x 256 (vector rows m), 8 waves (two per
// SIMD) of 128 x 64 (4 x 2 MFMA tiles), k slice 16 (one MFMA step per
// product).  The vector operand of a slice (from HBM) is loaded into
// registers two slices ahead (two register sets), the factor (from L2)
// one slice ahead, and both are split into one of two LDS stages one slice
// ahead, so every wait is on a register the compiler tracks exactly.  A stage
// holds six planes of 256 rows x 32 bytes (vector hi/mid/lo, factor
// hi/mid/lo); 16-byte chunk p of row rho holds k chunk p ^ sw(rho) with
// sw(rho) = (rho / 4 ^ rho / 8) % 2, which puts the fragment reads of every
// group of 16 lanes (and of 8) on distinct banks.

constexpr int XT = 512;                          // threads (8 waves)
constexpr int XKS = 16;                          // k slice
constexpr int XROW = 2 * XKS;                    // bytes of one plane row in LDS
constexpr int XPLANE = BM * XROW;                // bytes of one 256-row plane (8 KiB)
constexpr int XSTAGE = 6 * XPLANE;               // vector hi/mid/lo, then factor hi/mid/lo
constexpr int XLDS = 2 * XSTAGE;

// Workgroup barrier that orders LDS only: it waits for this wave's own LDS
// reads and writes (lgkmcnt) but not for global loads in flight, which a
// __syncthreads() fence would drain.  The memory clobber keeps the compiler
// from moving memory accesses across it.
__device__ inline void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Physical 16-byte chunk offset of logical chunk 0 in LDS row rho (see above).
__device__ inline int x3_swz(int rho) { return ((rho >> 2) ^ (rho >> 3)) & 1; }

__device__ inline floatx16 mfma_bf16(bf16x8 a, bf16x8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// v = h + m + l: each part the RNE BF16 rounding of what the earlier parts left.
// The remainders are exact in FP32 (each has at most 16 significant bits).
__device__ inline void split3(floatx4 v0, floatx4 v1, bf16x8& h, bf16x8& m, bf16x8& l) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float v = c < 4 ? v0[c] : v1[c - 4];
        const __bf16 hb = (__bf16)v;
        const float r1 = v - (float)hb;
        const __bf16 mb = (__bf16)r1;
        const float r2 = r1 - (float)mb;
        h[c] = hb;
        m[c] = mb;
        l[c] = (__bf16)r2;
    }
}

// One thread's share of a slice of the vector operand: 8 values (and for the direction pass
// the residual beside them), loaded two slices ahead (two register sets).
template <bool PNEW>
struct OpSet {
    floatx4 a[2];
    floatx4 r[PNEW ? 2 : 1];
};

// The same thread's 8 values of the factor (FP32, from L2), split like the vector operand
// when staged: loaded at the start of the step that stores them (one register set).  Two
// 16-byte loads instead of three pre-split planes: a third less L1 traffic for the factor,
// and fewer registers held across the step.
struct FacSet {
    floatx4 f[2];
};

// The direction pass (PNEW) leaves x += alpha p to the other passes: taking that step here (as
// the FP32 engine does) was measured slower, this pass being bound by its memory traffic.  With
// a second direction buffer (Gemm3Args::P2) p_old survives the direction pass, and the middle
// and last passes, bound by their MFMAs, each take the step on half of x: 4 elements per thread
// and k slice, loaded before the slice's MFMAs (after the factor, before the next slice's vector
// loads, so the latter stay in flight) and stored after them.
template <bool PNEW>
struct X3Thread {
    const float* A;      // this thread's vector row, at its k chunk
    const float* R;      // PNEW: residual
    float* P;            // PNEW: direction written back
    const float* F;      // this thread's factor row (FP32), at its k chunk
    float* XU;           // deferred step: this thread's 4 elements of x for k slice 0, else null
    const float* PU;     // p_old at the same elements
    float xalpha;
    double beta;
    uint32_t sdst;       // byte offset of this thread's chunk in a plane
    uint32_t afr, bfr;   // fragment offsets (factor tile 0, vector tile 0)

    __device__ __attribute__((always_inline)) void load(int k0, OpSet<PNEW>& o) const {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            o.a[h] = *(const floatx4*)(A + k0 + 4 * h);
            if constexpr (PNEW) o.r[h] = *(const floatx4*)(R + k0 + 4 * h);
        }
    }
    __device__ __attribute__((always_inline)) void load_fac(int k0, FacSet& fs) const {
        fs.f[0] = *(const floatx4*)(F + k0);
        fs.f[1] = *(const floatx4*)(F + k0 + 4);
    }
    // the direction is formed here, once per element (the direction pass has one N tile),
    // written back in place of p_old, then split into the stage
    __device__ __attribute__((always_inline)) void store(int k0, char* stage, const OpSet<PNEW>& o,
                                                         const FacSet& fs) const {
        floatx4 v[2] = {o.a[0], o.a[1]};
        if constexpr (PNEW) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
#pragma unroll
                for (int c = 0; c < 4; ++c) v[h][c] = pnew_of(o.r[h][c], v[h][c], beta);
                // streamed past the caches: no other pass of this MVM reads p before the last
                // pass's epilogue, and keeping it out of the L2 and the last-level cache leaves them
                // to the other passes' operands
                __builtin_nontemporal_store(v[h], (floatx4*)(P + k0 + 4 * h));
            }
        }
        bf16x8 hp, mp, lp;
        split3(v[0], v[1], hp, mp, lp);
        *(bf16x8*)(stage + sdst) = hp;
        *(bf16x8*)(stage + XPLANE + sdst) = mp;
        *(bf16x8*)(stage + 2 * XPLANE + sdst) = lp;
        split3(fs.f[0], fs.f[1], hp, mp, lp);
        *(bf16x8*)(stage + 3 * XPLANE + sdst) = hp;
        *(bf16x8*)(stage + 4 * XPLANE + sdst) = mp;
        *(bf16x8*)(stage + 5 * XPLANE + sdst) = lp;
    }
    // acc[i][j] += factor tile i x vector tile j over the slice: factor part outer, so only
    // one factor part's fragments are live at a time
    __device__ __attribute__((always_inline)) void compute(floatx16 (&acc)[4][2], const char* S) const {
        bf16x8 vv[3][2];
#pragma unroll
        for (int s = 0; s < 3; ++s)
#pragma unroll
            for (int j = 0; j < 2; ++j) vv[s][j] = *(const bf16x8*)(S + s * XPLANE + bfr + j * 32 * XROW);
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            bf16x8 fv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) fv[i] = *(const bf16x8*)(S + (3 + f) * XPLANE + afr + i * 32 * XROW);
            // factor part f meets vector parts 0 .. 2 - f: hh hm hl | mh mm | lh
#pragma unroll
            for (int s = 0; s < 3 - f; ++s)
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) acc[i][j] = mfma_bf16(fv[i], vv[s][j], acc[i][j]);
        }
    }
    // one k slice (the c-th): when LOAD start slice kl's loads into ld, multiply the slice in
    // stage S, when STORE split slice ks (held in st) into stage T; with XU take the deferred step
    // on the c-th chunk of this thread's share of x
    template <bool LOAD, bool STORE>
    __device__ __attribute__((always_inline)) void step(floatx16 (&acc)[4][2], const char* S, char* T,
                                                        OpSet<PNEW>& ld, const OpSet<PNEW>& st, int kl,
                                                        int ks, int c) const {
        FacSet fs;
        floatx4 xv = {}, pv = {};
        const int64_t xo = (int64_t)c * XT * 4;
        if constexpr (STORE) load_fac(ks, fs);
        if (XU) {                                          // streamed: read and written once
            xv = __builtin_nontemporal_load((const floatx4*)(XU + xo));
            pv = __builtin_nontemporal_load((const floatx4*)(PU + xo));
        }
        if constexpr (LOAD) load(kl, ld);
        __builtin_amdgcn_sched_barrier(0);                 // keep the loads ahead of the MFMAs
        compute(acc, S);
        if constexpr (STORE) store(ks, T, st, fs);
        if (XU) {
#pragma unroll
            for (int u = 0; u < 4; ++u) xv[u] = __builtin_fmaf(xalpha, pv[u], xv[u]);
            __builtin_nontemporal_store(xv, (floatx4*)(XU + xo));
        }
    }
};

template <bool PNEW, int EPI>
__global__ __launch_bounds__(XT) void k_gemm3x3(Gemm3Args a, PassDesc d) {
    __shared__ __attribute__((aligned(16))) char smem[XLDS];
    __shared__ double red[8];
    const int64_t rows = (int64_t)a.nrhs * d.rows_per_rhs;
    const int Mt = (int)(rows / BM), Nt = d.N / BN;
    const int L = xcd_linear(blockIdx.x, Mt * Nt);
    const int mt = L / Nt, nt = L % Nt;                    // N tiles of one row band run together
    const int64_t m0 = (int64_t)mt * BM;
    const int r = (int)(m0 / d.rows_per_rhs);
    if (a.gate && !a.gate[(int64_t)r * a.gate_stride]) return;
    const int n0 = nt * BN;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6) & 7;   // scalar, range known
    const int wn = wave >> 2, wm = wave & 3;               // factor rows wn*128.., vector rows wm*64..
    const int64_t K = d.K;
    // staging: thread t covers row t / 2, k chunk t % 2 (8 values) of each slice, of both operands
    const int srow = tid >> 1, schunk = tid & 1;
    const int64_t sofs = (m0 + srow) * K + 8 * schunk;
    // double-buffered direction (CG only): p_old in buffer pbuf, p_new in the other one
    const int cur = a.P2 ? a.cg[r].pbuf : 0;
    const float* const pold_b = cur ? a.P2 : a.X;
    float* const pnew_b = a.P2 ? (cur ? const_cast<float*>(a.X) : a.P2) : const_cast<float*>(a.X);
    X3Thread<PNEW> th;
    th.A = (PNEW ? pold_b : d.A) + sofs;
    th.R = PNEW ? d.R + sofs : nullptr;
    th.P = PNEW ? pnew_b + sofs : nullptr;
    th.F = d.B + (int64_t)(n0 + srow) * K + 8 * schunk;
    th.beta = PNEW ? a.cg[r].beta : 0.0;
    th.XU = nullptr;
    th.PU = nullptr;
    th.xalpha = 0.f;
    if constexpr (PNEW) {
        if (a.P2 && threadIdx.x == 0) {                    // every block stores the same values
            a.cg[r].pswap = 1;
            a.cg[r].xdefer = 1;
        }
    } else if (a.P2 && a.Xit && a.cg[r].xlag) {
        // the middle pass steps the first half of x, the last pass the second; each block its
        // 128 K elements of the half (one N tile per row band: every mode is 256)
        const int64_t nr = d.rows_per_rhs * K;
        const int64_t o = (int64_t)r * nr + (EPI == EPI_CG ? nr / 2 : 0) +
                          (m0 - (int64_t)r * d.rows_per_rhs) / 2 * K + 4 * tid;
        th.XU = a.Xit + o;
        th.PU = pold_b + o;
        th.xalpha = (float)a.cg[r].alpha;
    }
    th.sdst = (uint32_t)(srow * XROW + 16 * (schunk ^ x3_swz(srow)));
    // fragment reads: row (lane % 32) of each 32-row tile, logical chunk lane / 32
    const uint32_t flane = (uint32_t)((lane & 31) * XROW + 16 * ((lane >> 5) ^ x3_swz(lane & 31)));
    th.afr = flane + (uint32_t)(wn * 128 * XROW);
    th.bfr = flane + (uint32_t)(wm * 64 * XROW);

    floatx16 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx16{};

    char* const st0 = smem;
    char* const st1 = smem + XSTAGE;
    const int ns = (int)(K / XKS);                          // even and >= 16: K is a multiple of 256
    OpSet<PNEW> R0, R1;
    {
        FacSet fs;
        th.load_fac(0, fs);
        th.load(0, R0);
        th.load(XKS, R1);
        th.store(0, st0, R0, fs);
    }
    __syncthreads();
    // slice ks is multiplied from stage ks % 2 while slice ks + 2 loads into the register set slice
    // ks left free and slice ks + 1 is split into the other stage.  Every load and store inside the
    // loop is unconditional (the last two slices are peeled off), so the compiler's waits for the
    // register sets count exactly and the loads of slice ks + 2 stay in flight across the barrier.
    int ks = 0;
    for (; ks + 2 < ns; ks += 2) {
        th.template step<true, true>(acc, st0, st1, R0, R1, (ks + 2) * XKS, (ks + 1) * XKS, ks);
        lds_barrier();
        th.template step<true, true>(acc, st1, st0, R1, R0, (ks + 3) * XKS, (ks + 2) * XKS, ks + 1);
        lds_barrier();
    }
    th.template step<false, true>(acc, st0, st1, R0, R1, 0, (ks + 1) * XKS, ks);
    lds_barrier();
    th.template step<false, false>(acc, st1, st0, R1, R0, 0, 0, ks + 1);

    // epilogue straight from the accumulators: element v of tile (i, j) is output column
    // n0 + wn*128 + 32 i + row32(lane, v), entry (local row) + wm*64 + 32 j + lane % 32; the
    // column offset 8 (v / 4) + v % 4 is uniform, so every access is one per-lane pointer plus a
    // scalar offset
    const int64_t rpr = d.rows_per_rhs;
    const int64_t lane_pos = (int64_t)(n0 + wn * 128 + 4 * (lane >> 5)) * rpr +
                             (m0 - (int64_t)r * rpr) + wm * 64 + (lane & 31);
    float* const out = d.Out + (int64_t)r * d.N * rpr + lane_pos;
    // the last pass reads p_new (CG) or x (product)
    const float* const xin = EPI == EPI_STORE ? nullptr : pnew_b + (int64_t)r * d.N * rpr + lane_pos;
    const float* const dgv = a.dvec ? a.dvec + lane_pos : nullptr;
    const float s2 = (float)a.sigma2;
    double dacc[4] = {0.0, 0.0, 0.0, 0.0};                 // p.q in FP64, four short chains
    // the diagonal's presence is uniform: one branch around the whole epilogue
    auto epilogue = [&](auto has_diag) {
        constexpr bool HD = decltype(has_diag)::value;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                __builtin_amdgcn_sched_barrier(0);         // one tile's loads in flight at a time
                const int64_t t0 = (int64_t)(32 * i) * rpr + 32 * j;
                if constexpr (EPI == EPI_STORE) {
#pragma unroll
                    for (int v = 0; v < 16; ++v) out[t0 + (int64_t)(8 * (v >> 2) + (v & 3)) * rpr] = acc[i][j][v];
                } else {
#pragma unroll
                    for (int h = 0; h < 16; h += 8) {      // eight entries at a time
                        __builtin_amdgcn_sched_barrier(0);
                        float pv[8], dv[8];
#pragma unroll
                        for (int v = 0; v < 8; ++v) {
                            const int64_t o = t0 + (int64_t)(8 * ((h + v) >> 2) + (v & 3)) * rpr;
                            pv[v] = xin[o];                // p_new (CG) or x
                            dv[v] = HD ? dgv[o] : 0.f;
                        }
#pragma unroll
                        for (int v = 0; v < 8; ++v) {
                            const float q = acc[i][j][h + v] + (s2 + dv[v]) * pv[v];
                            if constexpr (EPI == EPI_CG)
                                dacc[v & 3] = __builtin_fma((double)pv[v], (double)q, dacc[v & 3]);
                            out[t0 + (int64_t)(8 * ((h + v) >> 2) + (v & 3)) * rpr] = q;
                        }
                    }
                }
            }
    };
    if (EPI != EPI_STORE && dgv) epilogue(std::true_type{});
    else epilogue(std::false_type{});
    if constexpr (EPI == EPI_CG) {
        const double sum = block_sum8((dacc[0] + dacc[1]) + (dacc[2] + dacc[3]), red);
        const int tpr = (int)(d.rows_per_rhs / BM) * Nt;
        const int t = (int)((m0 - (int64_t)r * d.rows_per_rhs) / BM) * Nt + nt;
        double tot;
        if (last_block_reduce8(sum, a.partials + (int64_t)r * a.part_stride, a.counters + r, tpr, t, &tot, red) &&
            threadIdx.x == 0) {
            CgState& st = a.cg[r];
            st.xlag = 0;                                   // the first pass has caught x up
            if (!(tot > 0.0) || !finite_d(tot)) {
                st.status = finite_d(tot) ? COLA_ERR_NOT_SPD : COLA_ERR_NONFINITE;
                st.active = 0;
                atomicSub(&a.cnt->num_active, 1);
            } else {
                st.alpha = st.rho / tot;
            }
        }
    }
}

}  // namespace

bool gemm3_supported(int prec, int Fv, int J, const int64_t* dims) {
    return (prec == COLA_PREC_FP32 || prec == COLA_PREC_BF16X3) && Fv == 3 && J == 1 && dims[0] >= BM && dims[1] >= BM && dims[0] % BM == 0 &&
           dims[1] % BM == 0 && dims[2] == BN;
}

hipError_t launch_gemm3(const Gemm3Args& a, int mode, hipStream_t s) {
    const int64_t dims[3] = {a.n1, a.n2, a.n3};
    if (!gemm3_supported(COLA_PREC_FP32, 3, 1, dims) || a.nrhs < 1) return hipErrorInvalidValue;
    const bool cg = a.epi == EPI_CG;
    if (cg && (!a.R || !a.cg || !a.partials || !a.counters)) return hipErrorInvalidValue;
    PassDesc d;
    std::memset(&d, 0, sizeof(d));
    if (mode == 3) {
        d.A = a.X; d.R = a.R; d.Pout = const_cast<float*>(a.X); d.B = a.K3; d.Out = a.Z1;
        d.rows_per_rhs = (int64_t)a.n1 * a.n2; d.K = a.n3; d.N = a.n3;
    } else if (mode == 2) {
        d.A = a.Z1; d.B = a.K2; d.Out = a.Z2;
        d.rows_per_rhs = (int64_t)a.n3 * a.n1; d.K = a.n2; d.N = a.n2;
    } else if (mode == 1) {
        d.A = a.Z2; d.B = a.K1; d.Out = a.Y;
        d.rows_per_rhs = (int64_t)a.n2 * a.n3; d.K = a.n1; d.N = a.n1;
    } else {
        return hipErrorInvalidValue;
    }
    const int64_t T = (int64_t)a.nrhs * d.rows_per_rhs / BM * (d.N / BN);
    if (a.bf16x3) {
        const dim3 grid((unsigned)T), block(XT);
        if (mode == 3 && cg) hipLaunchKernelGGL((k_gemm3x3<true, EPI_STORE>), grid, block, 0, s, a, d);
        else if (mode != 1) hipLaunchKernelGGL((k_gemm3x3<false, EPI_STORE>), grid, block, 0, s, a, d);
        else if (cg) hipLaunchKernelGGL((k_gemm3x3<false, EPI_CG>), grid, block, 0, s, a, d);
        else hipLaunchKernelGGL((k_gemm3x3<false, EPI_MATVEC>), grid, block, 0, s, a, d);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)T), block(kThreads);
    if (mode == 3 && cg) hipLaunchKernelGGL((k_gemm3<true, EPI_STORE>), grid, block, 0, s, a, d);
    else if (mode != 1) hipLaunchKernelGGL((k_gemm3<false, EPI_STORE>), grid, block, 0, s, a, d);
    else if (cg) hipLaunchKernelGGL((k_gemm3<false, EPI_CG>), grid, block, 0, s, a, d);
    else hipLaunchKernelGGL((k_gemm3<false, EPI_MATVEC>), grid, block, 0, s, a, d);
    return hipGetLastError();
}

}  // namespace cola
