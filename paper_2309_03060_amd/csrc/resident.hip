// Resident batched CG: many independent small systems in one persistent launch.
//
// CoLA solves blocks of right-hand sides together and stops when all have
// converged (App. D.5); here the block is a batch of independent systems
// K1 (x) K2 + diag(d) + sigma2 I of uneven sizes (mode sizes up to 128).
// Each (system, RHS) item is owned by one workgroup (16 waves) for as long as it
// iterates: its direction P and the intermediate T = P K2^T stay in LDS,
// x and r stay in registers laid out like the MFMA output of Q = K1 T, and
// the factors stream through LDS in 32-column chunks.  Workgroups pull items
// from an atomic queue ordered largest-first, so uneven iteration counts
// balance across the chip, and every workgroup leaves once the queue is
// empty.  An item leaves the kernel when its FP32 residual has dropped by
// delta (or converged): the FP64 residual kernel then folds x into the FP64
// solution, forms b - A x with the FP64 factors and replaces r, and the next
// round resumes the same CG (reliable updates).
#include "resident.h"

namespace cola {

constexpr int kResThreads = 1024;                // 16 waves per item
constexpr int RPS = kResMax + 4;                 // LDS row stride of P and T (floats)
constexpr int KC = 32;                           // factor columns staged per chunk
constexpr int FPS = KC + 4;                      // row stride of a factor chunk
constexpr int kResWaves = kResThreads / 64;
typedef float floatx16 __attribute__((ext_vector_type(16)));

// Sum over the 16 waves of an item's workgroup with a single barrier.  A
// caller that sums again must use another slot array (or pass a barrier)
// before it writes these slots again: other waves may still be reading them.
__device__ inline double block_sum16(double v, double* smem) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) smem[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kResThreads / 64; ++i) s += smem[i];
    return s;
}

__global__ __launch_bounds__(kThreads) void k_resident_prepare(ResArgs a, double tol, int max_iters, double delta) {
    __shared__ double red[4];
    const int item = blockIdx.x;
    const ResSys sy = a.sys[item / a.nrhs];
    const int rhs = item % a.nrhs;
    const int64_t base = (int64_t)a.nrhs * sy.vec_off + (int64_t)rhs * sy.n;
    double sb = 0.0, sr = 0.0;
    for (int64_t e = threadIdx.x; e < sy.n; e += kThreads) {
        const double v = a.b64[base + e];
        const float f = (float)v;
        a.r[base + e] = f;
        a.x[base + e] = 0.f;
        a.p[base + e] = 0.f;
        a.x64[base + e] = 0.0;
        sb += v * v;
        sr += (double)f * (double)f;
    }
    sb = block_sum(sb, red);
    sr = block_sum(sr, red);
    if (threadIdx.x == 0) {
        CgState& st = a.st[item];
        st.rho = sr;
        st.bnorm2 = sb;
        st.tol2 = tol * tol * sb;
        st.alpha = 0.0;
        st.beta = 0.0;
        st.iters = 0;
        st.max_iters = max_iters;
        st.delta = delta < 0.0 ? -delta : delta;
        st.restart_dir = delta < 0.0;
        st.rmax = sqrt(sr);
        st.rho_true = sb;
        st.need_update = 0;
        st.fails = 0;
        st.updates = 0;
        if (!finite_d(sb) || !finite_d(sr)) {
            st.status = COLA_ERR_NONFINITE;
            st.active = 0;
        } else if (sb <= st.tol2) {                 // b = 0: x = 0 after zero iterations
            st.status = COLA_OK;
            st.active = 0;
        } else {
            st.status = COLA_NOT_CONVERGED;
            st.active = 1;
            atomicAdd(&a.cnt->num_active, 1);
        }
    }
}

__global__ __launch_bounds__(kResThreads) void k_resident_cg(ResArgs a) {
    __shared__ __attribute__((aligned(16))) float Ps[kResMax * RPS];   // direction p
    __shared__ __attribute__((aligned(16))) float Ts[kResMax * RPS];   // T = P K2^T, then Q = K1 T
    __shared__ __attribute__((aligned(16))) float Fc[kResMax * FPS];   // factor chunk
    __shared__ double red_pq[kResWaves];       // slots of the p.q sums
    __shared__ double red_rr[kResWaves];       // slots of the r.r sums (every other barrier of the
                                               // iteration lies between one sum's reads and its next write)
    __shared__ int s_item;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lq = lane >> 4;
    // element ownership for the vector updates: 16 consecutive columns of one row
    const int orow = tid >> 3, ocol = (tid & 7) * 16;

    for (;;) {
        if (tid == 0) s_item = (int)atomicAdd(a.queue, 1u);
        __syncthreads();
        const int q = s_item;
        __syncthreads();
        if (q >= a.nitems) break;
        const int item = a.order[q];
        CgState* stp = &a.st[item];
        if (!stp->active) continue;
        const ResSys sy = a.sys[item / a.nrhs];
        const int rhs = item % a.nrhs;
        const int n1 = sy.n1, n2 = sy.n2;
        const int n1p = (n1 + 31) & ~31, n2p = (n2 + 31) & ~31;       // 32x32 MFMA tile extents
        const int n1k = n1p, n2k = n2p;                                 // K-loop extents (chunks of 32)
        const int tjn = n2p / 32;
        const int ntiles = (n1p / 32) * tjn;                            // <= 16: one tile per wave
        const bool has_tile = wave < ntiles;
        const int ti = has_tile ? 32 * (wave / tjn) : 0, tj = has_tile ? 32 * (wave % tjn) : 0;
        const int l32 = lane & 31, lh = lane >> 5;
        const int64_t base = (int64_t)a.nrhs * sy.vec_off + (int64_t)rhs * sy.n;
        const float* K1 = a.fac32 + sy.k1_off;
        const float* K2 = a.fac32 + sy.k2_off;
        const float* dgv = sy.diag_off >= 0 ? a.diag32 + sy.diag_off : nullptr;
        const float s2 = (float)sy.sigma2;
        const bool own = orow < n1;
        const int ncol = own ? (n2 - ocol < 16 ? (n2 - ocol > 0 ? n2 - ocol : 0) : 16) : 0;
        float* xo = a.x + base + (int64_t)orow * n2 + ocol;     // owned x (global, updated in place)
        const float* dgo = dgv ? dgv + orow * n2 + ocol : nullptr;
        float* po = Ps + orow * RPS + ocol;
        float* qo = Ts + orow * RPS + ocol;

        // scalars (read by every thread; only thread 0 writes them back)
        double rho = stp->rho, beta = stp->beta;
        const double tol2 = stp->tol2, delta = stp->delta, rmax = stp->rmax;
        int iters = stp->iters;
        const int max_iters = stp->max_iters;
        int status = stp->status, active = 1, need_update = 0;

        // zero the LDS tiles over the full K-loop extent, then load p and r
        for (int e = tid; e < n1k * RPS; e += kResThreads) {
            Ps[e] = 0.f;
            Ts[e] = 0.f;
        }
        __syncthreads();
        for (int e = tid; e < n1 * n2; e += kResThreads) Ps[(e / n2) * RPS + (e % n2)] = a.p[base + e];
        float rr[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) rr[j] = j < ncol ? a.r[base + (int64_t)orow * n2 + ocol + j] : 0.f;
        __syncthreads();

        // Factor chunks in the order the iteration consumes them (K2 column
        // chunks, then K1 column chunks, then K2 again for the next iteration):
        // every thread holds its four entries of the next chunk in registers,
        // loaded while the current chunk's MFMAs run.  Entry u of a chunk is
        // e = tid + u * kResThreads, row e / KC, column e % KC of the chunk.
        const int nc2 = n2k / KC, nc1 = n1k / KC;
        int cnext = 0;                                  // chunk the registers hold
        float fpre[4];
        auto fetch = [&](int c) {
            const bool second = c >= nc2;
            const float* K = second ? K1 : K2;
            const int nk = second ? n1 : n2;
            const int npad = second ? n1p : n2p;
            const int c0 = (second ? c - nc2 : c) * KC;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = tid + u * kResThreads, rb = e / KC, kc = e % KC;
                fpre[u] = (e < npad * KC && rb < nk && c0 + kc < nk) ? K[rb * nk + c0 + kc] : 0.f;
            }
        };
        auto fetch_next = [&]() {
            cnext = cnext + 1 == nc2 + nc1 ? 0 : cnext + 1;
            fetch(cnext);
        };
        auto stage_chunk = [&](int npad) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = tid + u * kResThreads;
                if (e < npad * KC) Fc[(e / KC) * FPS + e % KC] = fpre[u];
            }
        };
        fetch(0);

        for (;;) {
            // p = r + beta p on the owned elements
            const float bf = (float)beta;
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (j < ncol) po[j] = __builtin_fmaf(bf, po[j], rr[j]);
            __syncthreads();
            // T = P K2^T   (32x32 tile per wave: T[ti.., tj..] = sum_l P[ti.., l] K2[tj.., l])
            floatx16 acc;
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[v] = 0.f;
            for (int l0 = 0; l0 < n2k; l0 += KC) {
                stage_chunk(n2p);
                __syncthreads();
                fetch_next();                               // lands during this chunk's MFMAs
                if (has_tile) {
                    const float* pa = Ps + (ti + l32) * RPS + l0 + lh;
                    const float* fb = Fc + (tj + l32) * FPS + lh;
#pragma unroll 4
                    for (int kk = 0; kk < KC; kk += 2)
                        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(pa[kk], fb[kk], acc, 0, 0, 0);
                }
                __syncthreads();
            }
            if (has_tile)
#pragma unroll
                for (int v = 0; v < 16; ++v)
                    Ts[(ti + 8 * (v >> 2) + 4 * lh + (v & 3)) * RPS + tj + l32] = acc[v];
            __syncthreads();
            // Q = K1 T   (Q[ti.., tj..] = sum_i K1[ti.., i] T[i, tj..])
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[v] = 0.f;
            for (int i0 = 0; i0 < n1k; i0 += KC) {
                stage_chunk(n1p);
                __syncthreads();
                fetch_next();
                if (has_tile) {
                    const float* fa = Fc + (ti + l32) * FPS + lh;
                    const float* tb = Ts + (i0 + lh) * RPS + tj + l32;
#pragma unroll 4
                    for (int kk = 0; kk < KC; kk += 2)
                        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[kk], tb[kk * RPS], acc, 0, 0, 0);
                }
                __syncthreads();
            }
            // stage Q over the dead T tile, then the owned-element epilogue
            if (has_tile)
#pragma unroll
                for (int v = 0; v < 16; ++v)
                    Ts[(ti + 8 * (v >> 2) + 4 * lh + (v & 3)) * RPS + tj + l32] = acc[v];
            __syncthreads();
            // q = K1 T + (sigma2 + d) p;  mu = p.q
            double mu_l = 0.0;
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (j < ncol) {
                    const float pe = po[j];
                    const float qv = qo[j] + (s2 + (dgo ? dgo[j] : 0.f)) * pe;
                    qo[j] = qv;
                    mu_l += (double)pe * (double)qv;
                }
            const double mu = block_sum16(mu_l, red_pq);
            if (!(mu > 0.0) || !finite_d(mu)) {
                status = finite_d(mu) ? COLA_ERR_NOT_SPD : COLA_ERR_NONFINITE;
                active = 0;
                break;
            }
            const float af = (float)(rho / mu);
            double rho_l = 0.0;
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (j < ncol) {
                    xo[j] = __builtin_fmaf(af, po[j], xo[j]);
                    rr[j] = __builtin_fmaf(-af, qo[j], rr[j]);
                    rho_l += (double)rr[j] * (double)rr[j];
                }
            const double rn = block_sum16(rho_l, red_rr);
            ++iters;
            bool stop = false;
            if (!finite_d(rn)) {
                status = COLA_ERR_NONFINITE;
                active = 0;
                stop = true;
            } else if (rn <= tol2) {                 // pause; the FP64 residual decides
                need_update = 1;
                active = 0;
                stop = true;
            } else if (iters >= max_iters) {
                status = COLA_NOT_CONVERGED;
                active = 0;
                stop = true;
            } else if (rn < delta * delta * rmax * rmax) {
                need_update = 1;
                stop = true;
            }
            beta = rn / rho;
            rho = rn;
            if (stop) break;
        }
        // write the state back
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (j < ncol) a.r[base + (int64_t)orow * n2 + ocol + j] = rr[j];
        for (int e = tid; e < n1 * n2; e += kResThreads) a.p[base + e] = Ps[(e / n2) * RPS + (e % n2)];
        if (tid == 0) {
            stp->rho = rho;
            stp->beta = beta;
            stp->iters = iters;
            stp->status = status;
            stp->need_update = need_update;
            if (!active) {
                stp->active = 0;
                atomicSub(&a.cnt->num_active, 1);
            }
        }
        __syncthreads();
    }
}

// FP64 residual of requested items: fold the FP32 iterate into the FP64
// solution, r = b - (K1 X K2^T + (sigma2 + d) x) with the FP64 factors,
// r_lo = r; then the reliable-update decision.  Final pass (a.all_items):
// every item without a certified residual (status not OK); a converged item
// was certified by its last update and its x has not changed since.
// Both mode products run on the FP64 matrix cores (v_mfma_f64_16x16x4f64;
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16], accumulator
// element v sits at row 4 v + l / 16, column l % 16).  X stays in LDS (padded rows, zero beyond the system), the factors
// and T = X K2^T come from L2.  Each wave computes groups of 1 x 4 output
// tiles (16 x 64) that share the A fragment; 16 waves per item so that four
// waves per SIMD cover each other's L2 latency.
constexpr int kResidThreads = 1024;
constexpr int PX = kResMax + 2;                  // pitch of X: conflict-free A-operand reads

__device__ inline doublex4 mma_f64(double a, double b, doublex4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(kResidThreads) void k_resident_resid64(ResArgs a) {
    __shared__ double Xs[kResMax * PX];
    __shared__ double red[kResWaves];
    const int item = blockIdx.x;
    CgState& st = a.st[item];
    if (a.all_items ? st.status == COLA_OK : !st.need_update) return;
    const ResSys sy = a.sys[item / a.nrhs];
    const int rhs = item % a.nrhs;
    const int n1 = sy.n1, n2 = sy.n2;
    const int64_t base = (int64_t)a.nrhs * sy.vec_off + (int64_t)rhs * sy.n;
    const double* K1 = a.fac64 + sy.k1_off;
    const double* K2 = a.fac64 + sy.k2_off;
    const double* dgv = sy.diag_off >= 0 ? a.diag64 + sy.diag_off : nullptr;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const int n1p = (n1 + 15) & ~15, n2p = (n2 + 15) & ~15;       // 16 x 16 tile extents
    // fold the FP32 correction into x64 and stage X (zero in the padding)
    for (int e = tid; e < n1p * n2p; e += kResidThreads) {
        const int row = e / n2p, col = e % n2p;
        double v = 0.0;
        if (row < n1 && col < n2) {
            const int64_t g = base + (int64_t)row * n2 + col;
            v = a.x64[g] + (double)a.x[g];
            a.x64[g] = v;
            a.x[g] = 0.f;
        }
        Xs[row * PX + col] = v;
    }
    __syncthreads();
    const int nt1 = n1p / 16, nt2 = n2p / 16, ng2 = (nt2 + 3) / 4;
    // T[i][j] = sum_l X[i][l] K2[j][l]
    for (int g = wave; g < nt1 * ng2; g += kResWaves) {
        const int i0 = (g / ng2) * 16, j0 = (g % ng2) * 64;
        doublex4 acc[4] = {};
        for (int k = 0; k < n2p; k += 4) {
            const int kk = k + lk;
            const double av = Xs[(i0 + lr) * PX + kk];
            double bv[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int col = j0 + 16 * t + lr;
                bv[t] = (col < n2 && kk < n2) ? K2[(int64_t)col * n2 + kk] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] = mma_f64(av, bv[t], acc[t]);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = i0 + 4 * v + lk, col = j0 + 16 * t + lr;
                if (row < n1 && col < n2) a.t64[base + (int64_t)row * n2 + col] = acc[t][v];
            }
    }
    __syncthreads();                                    // T complete
    // q = K1 T + (sigma2 + d) x,  r = b - q
    double rr = 0.0;
    for (int g = wave; g < nt1 * ng2; g += kResWaves) {
        const int i0 = (g / ng2) * 16, j0 = (g % ng2) * 64;
        doublex4 acc[4] = {};
        const int arow = i0 + lr;
        for (int k = 0; k < n1p; k += 4) {
            const int kk = k + lk;
            const double av = (arow < n1 && kk < n1) ? K1[(int64_t)arow * n1 + kk] : 0.0;
            double bv[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int col = j0 + 16 * t + lr;
                bv[t] = (col < n2 && kk < n1) ? a.t64[base + (int64_t)kk * n2 + col] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] = mma_f64(av, bv[t], acc[t]);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = i0 + 4 * v + lk, col = j0 + 16 * t + lr;
                if (row < n1 && col < n2) {
                    const int64_t e = (int64_t)row * n2 + col;
                    const double dg = sy.sigma2 + (dgv ? dgv[e] : 0.0);
                    const double rv = a.b64[base + e] - (acc[t][v] + dg * Xs[row * PX + col]);
                    a.r[base + e] = (float)rv;
                    rr += rv * rv;
                }
            }
    }
    rr = block_sum16(rr, red);
    if (tid == 0) {
        st.rho_true = rr;
        if (!a.all_items) reliable_finish(st, a.cnt);
    }
}

hipError_t launch_resident_prepare(const ResArgs& a, double tol, int max_iters, double delta, hipStream_t s) {
    hipLaunchKernelGGL(k_resident_prepare, dim3(a.nitems), dim3(kThreads), 0, s, a, tol, max_iters, delta);
    return hipGetLastError();
}
hipError_t launch_resident_cg(const ResArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_resident_cg, dim3(grid), dim3(kResThreads), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_resident_resid64(const ResArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_resident_resid64, dim3(a.nitems), dim3(kResidThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace cola
