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

}  // namespace

bool gemm3_supported(int prec, int Fv, int J, const int64_t* dims) {
    return prec == COLA_PREC_FP32 && Fv == 3 && J == 1 && dims[0] >= BM && dims[1] >= BM && dims[0] % BM == 0 &&
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
    const dim3 grid((unsigned)T), block(kThreads);
    if (mode == 3 && cg) hipLaunchKernelGGL((k_gemm3<true, EPI_STORE>), grid, block, 0, s, a, d);
    else if (mode != 1) hipLaunchKernelGGL((k_gemm3<false, EPI_STORE>), grid, block, 0, s, a, d);
    else if (cg) hipLaunchKernelGGL((k_gemm3<false, EPI_CG>), grid, block, 0, s, a, d);
    else hipLaunchKernelGGL((k_gemm3<false, EPI_MATVEC>), grid, block, 0, s, a, d);
    return hipGetLastError();
}

}  // namespace cola
