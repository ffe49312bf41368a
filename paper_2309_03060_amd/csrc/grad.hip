// Adjoint backward of the solve, and the contraction-tile autotuner.
//
// App. B.2 (autograd rule 1): with lambda = A^{-1} dL/dx, the gradient of the
// loss with respect to any operator parameter theta is
//     -sum_r lambda_r^T (dA/dtheta) x_r.
// For a factor K_jk of a Kronecker term this is a contraction of the mode-k
// unfoldings of Lambda and of Z = X multiplied along every other mode by the
// term's factors:  dK_jk = -sum_r Lambda_r,(k) Z_r,(k)^T  (n_k x n_k), a GEMM
// whose inner dimension is nrhs * n / n_k.  It runs as a split-K FP64 MFMA
// kernel (each block a slice of the inner dimension), and a second kernel
// sums the slices in fixed order.  The diagonal and sigma2 gradients are
// -sum_r lambda_r * x_r and its total.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "grad.h"

#include "gemm.h"
#include "gemm3.h"
#include "vector.h"

namespace cola {

// partial[c][a][i] = sum over g in slice c and t of L[g, a, t] * Z[g, i, t]
template <int WM, int WN, bool TRAIL1>
__global__ __launch_bounds__(kThreads) void k_grad_gemm(const double* L, const double* Z, int64_t G, int nk,
                                                        int64_t T, int64_t g_per_chunk, double* partial) {
    constexpr int MT = 32 * WM, NT = 32 * WN, KT = 16, KP = KT + 2;
    __shared__ double As[MT * KP];
    __shared__ double Bs[NT * KP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int nNt = (nk + NT - 1) / NT;
    const int64_t a0 = (int64_t)(blockIdx.x / nNt) * MT;
    const int64_t i0 = (int64_t)(blockIdx.x % nNt) * NT;
    const int64_t c = blockIdx.y;
    const int64_t gbeg = c * g_per_chunk;
    const int64_t gend = (gbeg + g_per_chunk < G) ? gbeg + g_per_chunk : G;

    doublex4 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = doublex4{0, 0, 0, 0};

    auto compute = [&]() {
#pragma unroll
        for (int kk = 0; kk < KT; kk += 4) {
            double av[WM], bv[WN];
#pragma unroll
            for (int i = 0; i < WM; ++i) av[i] = As[(wm * WM * 16 + i * 16 + (lane & 15)) * KP + kk + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < WN; ++j) bv[j] = Bs[(wn * WN * 16 + j * 16 + (lane & 15)) * KP + kk + (lane >> 4)];
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
    };

    if constexpr (TRAIL1) {
        // inner index = g; rows L[g, :] contiguous along a
        for (int64_t k0 = gbeg; k0 < gend; k0 += KT) {
            for (int e = tid; e < MT * KT; e += kThreads) {
                const int m = e % MT, k = e / MT;
                const int64_t gg = k0 + k, aa = a0 + m;
                As[m * KP + k] = (gg < gend && aa < nk) ? L[gg * nk + aa] : 0.0;
            }
            for (int e = tid; e < NT * KT; e += kThreads) {
                const int m = e % NT, k = e / NT;
                const int64_t gg = k0 + k, ii = i0 + m;
                Bs[m * KP + k] = (gg < gend && ii < nk) ? Z[gg * nk + ii] : 0.0;
            }
            __syncthreads();
            compute();
            __syncthreads();
        }
    } else {
        for (int64_t g = gbeg; g < gend; ++g) {
            const double* Lg = L + g * nk * T;
            const double* Zg = Z + g * nk * T;
            for (int64_t t0 = 0; t0 < T; t0 += KT) {
                for (int e = tid; e < MT * KT; e += kThreads) {
                    const int m = e / KT, k = e % KT;
                    const int64_t tt = t0 + k, aa = a0 + m;
                    As[m * KP + k] = (tt < T && aa < nk) ? Lg[aa * T + tt] : 0.0;
                }
                for (int e = tid; e < NT * KT; e += kThreads) {
                    const int m = e / KT, k = e % KT;
                    const int64_t tt = t0 + k, ii = i0 + m;
                    Bs[m * KP + k] = (tt < T && ii < nk) ? Zg[ii * T + tt] : 0.0;
                }
                __syncthreads();
                compute();
                __syncthreads();
            }
        }
    }
    double* out = partial + c * (int64_t)nk * nk;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t a = a0 + wm * WM * 16 + i * 16 + acc_row(acc[i][j][v], lane, v);
                const int64_t ii = i0 + wn * WN * 16 + j * 16 + (lane & 15);
                if (a < nk && ii < nk) out[a * nk + ii] = acc[i][j][v];
            }
}

// dK = scale * (-sum_c partial[c])
__global__ void k_grad_reduce(const double* partial, int64_t nchunks, int64_t nn, double* dK, double scale) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int64_t c = 0; c < nchunks; ++c) s += partial[c * nn + e];
        dK[e] = -s * scale;
    }
}

// dd[e] = scale * (-sum_r lambda_r[e] x_r[e]);  dsigma2 = scale * (-sum_e sum_r lambda_r[e] x_r[e])
__global__ __launch_bounds__(kThreads) void k_grad_diag(const double* X, const double* Lam, int64_t n, int nrhs,
                                                        double* dd, double* dsigma2, double* partials,
                                                        uint32_t* counter, double scale) {
    __shared__ double red[4];
    double tot_local = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += (int64_t)gridDim.x * kThreads) {
        double s = 0.0;
        for (int r = 0; r < nrhs; ++r) s += Lam[(int64_t)r * n + e] * X[(int64_t)r * n + e];
        if (dd) dd[e] = -s * scale;
        tot_local += s;
    }
    const double b = block_sum(tot_local, red);
    double tot;
    if (last_block_reduce(b, partials, counter, gridDim.x, blockIdx.x, &tot, red) && threadIdx.x == 0 && dsigma2)
        *dsigma2 = -tot * scale;
}

// ---------------------------------------------------------------------------
int32_t apply_modes_f64(cola_op_s* op, const SysInfo& s, int term, int skip, const double* X, int nrhs,
                        double* out, hipStream_t st) {
    // ping-pong between out and inter[1]; the final product lands in `out`
    std::vector<int> modes;
    for (int m = s.Fv - 1; m >= 0; --m)
        if (m != skip && !(s.F == 1 && m == 0)) modes.push_back(m);
    if (modes.empty()) {
        if (hipMemcpyAsync(out, X, sizeof(double) * (size_t)nrhs * s.n, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return COLA_ERR_HIP;
        return COLA_OK;
    }
    double* bufs[2] = {out, (double*)op->ws.inter[1]};
    int cur = (modes.size() % 2 == 1) ? 0 : 1;  // so that the last pass writes `out`
    const double* in = X;
    for (size_t q = 0; q < modes.size(); ++q) {
        const int m = modes[q];
        const int64_t nk = s.dims[m];
        int64_t lead = 1, trail = 1;
        for (int u = 0; u < m; ++u) lead *= s.dims[u];
        for (int u = m + 1; u < s.Fv; ++u) trail *= s.dims[u];
        PassArgs a;
        std::memset(&a, 0, sizeof(a));
        a.nk = (int32_t)nk;
        a.nsum = 1;
        a.nout = 1;
        a.K = op->fac64 + s.fac_off[m] + (int64_t)term * nk * nk;
        a.k_tstride = nk * nk;
        a.X = in;
        a.Y = bufs[cur];
        a.epi = EPI_STORE;
        const bool rows = (trail == 1);
        a.G = (int64_t)nrhs * lead;
        a.B = rows ? 1 : trail;
        a.a_per_rhs = lead;
        TileCfg cfg{nk >= 64 ? 2 : 1, rows ? (nk >= 64 ? 2 : 1) : (trail >= 64 ? 2 : 1)};
        if (rows) cfg.wm = 2;
        if (launch_contract(COLA_PREC_FP64, rows, a, cfg, st) != hipSuccess) return COLA_ERR_HIP;
        in = bufs[cur];
        cur ^= 1;
    }
    return COLA_OK;
}

int32_t grad_system(cola_op_s* op, const SysInfo& s, const double* X, const double* Lam, int nrhs,
                    void* const* dfactors, void* ddiag, double* dsigma2, hipStream_t st, double scale) {
    if (op->ws.nrhs < nrhs) return COLA_ERR_INVALID_ARG;    // staging buffers must hold nrhs vectors
    if (dfactors) {
        double* Z = (double*)op->ws.inter[0];
        for (int j = 0; j < s.J; ++j)
            for (int k = 0; k < s.F; ++k) {
                double* dK = (double*)dfactors[j * s.F + k];
                if (!dK) continue;
                const int kv = (s.F == 1) ? 1 : k;
                int32_t rc = apply_modes_f64(op, s, j, kv, X, nrhs, Z, st);
                if (rc != COLA_OK) return rc;
                const int64_t nk = s.dims[kv];
                int64_t lead = 1, trail = 1;
                for (int u = 0; u < kv; ++u) lead *= s.dims[u];
                for (int u = kv + 1; u < s.Fv; ++u) trail *= s.dims[u];
                const int64_t G = (int64_t)nrhs * lead;
                const int wm = nk >= 64 ? 2 : 1, wn = wm;
                const int64_t tiles = ((nk + 32 * wm - 1) / (32 * wm)) * ((nk + 32 * wn - 1) / (32 * wn));
                int64_t chunks = std::max<int64_t>(1, 1024 / tiles);
                if (trail == 1) chunks = std::min<int64_t>(chunks, (G + 15) / 16);
                chunks = std::min<int64_t>(chunks, G);
                const int64_t gpc = (G + chunks - 1) / chunks;
                chunks = (G + gpc - 1) / gpc;
                // partial slices live in the last workspace vector buffer when they fit, else a grown buffer
                double* partial = nullptr;
                const size_t need = (size_t)chunks * nk * nk;
                const size_t have = (size_t)op->ws.nrhs * op->nmax;
                if (need <= have) {
                    partial = (double*)op->ws.vq;
                } else {
                    if (op->grad_buf_elems < need) {
                        dev_free(op, op->grad_buf);
                        op->grad_buf = nullptr;
                        op->grad_buf_elems = 0;
                        if (dev_alloc(op, (void**)&op->grad_buf, need * sizeof(double)) != COLA_OK) return COLA_ERR_OOM;
                        op->grad_buf_elems = need;
                    }
                    partial = op->grad_buf;
                }
                dim3 grid((unsigned)tiles, (unsigned)chunks);
                if (wm == 2) {
                    if (trail == 1)
                        hipLaunchKernelGGL((k_grad_gemm<2, 2, true>), grid, dim3(kThreads), 0, st, Lam, Z, G, (int)nk,
                                           trail, gpc, partial);
                    else
                        hipLaunchKernelGGL((k_grad_gemm<2, 2, false>), grid, dim3(kThreads), 0, st, Lam, Z, G, (int)nk,
                                           trail, gpc, partial);
                } else {
                    if (trail == 1)
                        hipLaunchKernelGGL((k_grad_gemm<1, 1, true>), grid, dim3(kThreads), 0, st, Lam, Z, G, (int)nk,
                                           trail, gpc, partial);
                    else
                        hipLaunchKernelGGL((k_grad_gemm<1, 1, false>), grid, dim3(kThreads), 0, st, Lam, Z, G, (int)nk,
                                           trail, gpc, partial);
                }
                if (hipGetLastError() != hipSuccess) return COLA_ERR_HIP;
                const int64_t nn = nk * nk;
                hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)std::min<int64_t>((nn + 255) / 256, 4096)), dim3(256),
                                   0, st, partial, chunks, nn, dK, scale);
                if (hipGetLastError() != hipSuccess) return COLA_ERR_HIP;
            }
    }
    if (ddiag || dsigma2) {
        const unsigned blocks = (unsigned)std::min<int64_t>(512, std::max<int64_t>(1, (s.n + 2047) / 2048));
        hipLaunchKernelGGL(k_grad_diag, dim3(blocks), dim3(kThreads), 0, st, X, Lam, s.n, nrhs, (double*)ddiag,
                           dsigma2, op->ws.partials, op->ws.counters, scale);
        if (hipGetLastError() != hipSuccess) return COLA_ERR_HIP;
    }
    return COLA_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: for each contraction pass of each system (at this nrhs), time
// every tile candidate over a few launches with HIP events and keep the
// fastest in the op's tile table.
int32_t autotune_op(cola_op_s* op, int nrhs, hipStream_t st) {
    int32_t rc = ensure_workspace(op, nrhs, st);
    if (rc != COLA_OK) return rc;
    const TileCfg cands[] = {{1, 1}, {1, 2}, {2, 1}, {2, 2}, {4, 2}, {2, 4}, {4, 4}, {1, 4}, {4, 1}};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return COLA_ERR_HIP;
    std::vector<int> precs = {COLA_PREC_FP64};
    if (op->prec != COLA_PREC_FP64) precs.push_back(op->prec);
    for (const SysInfo& s : op->sys) {
        for (int prec : precs) {
            if ((op->use_gemm2 && gemm2_supported(prec, s.Fv, s.dims)) ||
                (op->use_gemm3 && gemm3_supported(prec, s.Fv, s.J, s.dims)))
                continue;                                                         // fixed GEMM tiles
            for (int k = s.Fv - 1; k >= 0; --k) {
                const int64_t nk = s.dims[k];
                int64_t lead = 1, trail = 1;
                for (int u = 0; u < k; ++u) lead *= s.dims[u];
                for (int u = k + 1; u < s.Fv; ++u) trail *= s.dims[u];
                const bool rows = (k == s.Fv - 1);
                PassKey key{prec, rows ? 1 : 0, nk, rows ? 1 : trail, lead};
                float best = 1e30f;
                TileCfg bestc = cands[1];
                for (const TileCfg& c : cands) {
                    PassArgs a;
                    std::memset(&a, 0, sizeof(a));
                    a.nk = (int32_t)nk;
                    a.nsum = (k == 0) ? s.J : 1;
                    a.nout = (k == 0) ? 1 : s.J;
                    a.G = (int64_t)nrhs * lead;
                    a.B = rows ? 1 : trail;
                    a.a_per_rhs = lead;
                    a.X = op->ws.vx;
                    a.x_tstride = 0;
                    a.Y = op->ws.inter[0];
                    a.y_tstride = (int64_t)nrhs * s.n;
                    a.K = (prec == COLA_PREC_FP64) ? (const void*)(op->fac64 + s.fac_off[k])
                          : (prec == COLA_PREC_FP32) ? (const void*)(op->fac32 + s.fac_off[k])
                                                     : (const void*)(op->facbf + s.fac_off[k]);
                    a.k_tstride = nk * nk;
                    a.k_plane = op->fac_elems;
                    a.epi = EPI_STORE;
                    if (launch_contract(prec, rows, a, c, st) != hipSuccess) return COLA_ERR_HIP;  // warm
                    (void)hipEventRecord(e0, st);
                    for (int rep = 0; rep < 5; ++rep)
                        if (launch_contract(prec, rows, a, c, st) != hipSuccess) return COLA_ERR_HIP;
                    (void)hipEventRecord(e1, st);
                    if (hipEventSynchronize(e1) != hipSuccess) return COLA_ERR_HIP;
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    if (ms < best) {
                        best = ms;
                        bestc = c;
                    }
                }
                op->tiles[key] = bestc;
                if (std::getenv("COLA_VERBOSE"))
                    std::fprintf(stderr, "cola_autotune: prec %d %s nk %lld B %lld lead %lld -> tile %dx%d (%.1f us)\n",
                                 prec, rows ? "rows" : "cols", (long long)nk, (long long)(rows ? 1 : trail),
                                 (long long)lead, 32 * bestc.wm, 32 * bestc.wn, 1e3 * best / 5);
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    op->tiles_version += 1;
    return COLA_OK;
}

}  // namespace cola
