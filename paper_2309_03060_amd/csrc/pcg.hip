// Exact diagonals of sum-of-Kronecker-plus-diagonal operators, the vector
// phase of preconditioned CG, and the accumulation of probe estimators.
//
// Diag(A + B) = Diag(A) + Diag(B) and Diag(A (x) B) = vec(Diag(A) Diag(B)^T)
// (App. A, diagonal rules): entry i of a Kronecker term with multi-index
// (i1, i2, i3) is the product of the factors' diagonal entries, so the whole
// diagonal costs O(n J F) reads of factor diagonals (cached) and one write per
// entry.  Preconditioned CG follows the textbook recurrence: after the step
// x += alpha p, r -= alpha q the residual norm decides convergence, then
// z = M^{-1} r, rho' = r.z, beta = rho' / rho, and the next MVM pass forms
// p = z + beta p.  The probe estimators of Diag(A) average z . A z over probes
// (Sec. 3.3; App. B.1 for the doubly stochastic variant over the terms of a
// Sum).
#include "pcg.h"

namespace cola {
namespace {

__device__ inline double diag_entry(const DiagArgs& a, int64_t i) {
    int64_t idx[3] = {0, 0, 0};
    int64_t rem = i;
    for (int k = a.F - 1; k >= 0; --k) {
        idx[k] = rem % a.dims[k];
        rem /= a.dims[k];
    }
    double v = a.sigma2 + (a.dvec ? a.dvec[i] : 0.0);
    for (int j = 0; j < a.J; ++j) {
        double t = 1.0;
        for (int k = 0; k < a.F; ++k) {
            const int64_t nk = a.dims[k];
            t *= a.fac[k][(int64_t)j * nk * nk + idx[k] * nk + idx[k]];
        }
        v += t;
    }
    return v;
}

__global__ __launch_bounds__(kThreads) void k_kron_diagonal(DiagArgs a, double* out, int invert) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * kThreads) {
        const double v = diag_entry(a, i);
        out[i] = invert ? 1.0 / v : v;
    }
}

// one block: the trace-matching shift of the Kronecker-eigen preconditioner
__global__ __launch_bounds__(kThreads) void k_trace_shift(DiagArgs a, double* out) {
    __shared__ double red[4];
    double s = 0.0;
    if (a.dvec)
        for (int64_t i = threadIdx.x; i < a.n; i += kThreads) s += a.dvec[i];
    s = block_sum(s, red);
    double c = a.sigma2 + s / (double)a.n;
    for (int j = 1; j < a.J; ++j) {
        double prod = 1.0;
        for (int k = 0; k < a.F; ++k) {
            const int64_t nk = a.dims[k];
            double t = 0.0;
            for (int64_t d = threadIdx.x; d < nk; d += kThreads) t += a.fac[k][(int64_t)j * nk * nk + d * nk + d];
            t = block_sum(t, red);
            prod *= t / (double)nk;
        }
        c += prod;
    }
    if (threadIdx.x == 0) *out = c;
}

__global__ __launch_bounds__(kThreads) void k_pcg_update(double* x, double* r, const double* p, const double* q,
                                                         int64_t n, CgState* cg, double* partials, int part_stride,
                                                         uint32_t* counters, SolveCounters* cnt, ResHist rh) {
    __shared__ double red[4];
    const int64_t g = blockIdx.y;
    if (!cg[g].active) return;
    const double alpha = cg[g].alpha;
    double* xg = x + g * n;
    double* rg = r + g * n;
    const double* pg = p + g * n;
    const double* qg = q + g * n;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        xg[i] = fma(alpha, pg[i], xg[i]);
        const double rv = fma(-alpha, qg[i], rg[i]);
        rg[i] = rv;
        s += rv * rv;
    }
    s = block_sum(s, red);
    double tot;
    if (last_block_reduce(s, partials + g * part_stride, counters + g, gridDim.x, blockIdx.x, &tot, red) &&
        threadIdx.x == 0) {
        CgState& st = cg[g];
        st.iters += 1;
        st.rho_true = tot;                          // r.r (rho holds r.z)
        record_residual(rh, g, st, tot);
        bool stop = true;
        if (!finite_d(tot)) st.status = COLA_ERR_NONFINITE;
        else if (tot <= st.tol2) st.status = COLA_OK;
        else if (st.iters >= st.max_iters) st.status = COLA_NOT_CONVERGED;
        else stop = false;
        if (stop) {
            st.active = 0;
            atomicSub(&cnt->num_active, 1);
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_pcg_precond_dot(const double* r, double* z, const double* dinv,
                                                              int64_t n, CgState* cg, double* partials,
                                                              int part_stride, uint32_t* counters,
                                                              SolveCounters* cnt) {
    __shared__ double red[4];
    const int64_t g = blockIdx.y;
    if (!cg[g].active) return;
    const double* rg = r + g * n;
    double* zg = z + g * n;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const double rv = rg[i];
        double zv;
        if (dinv) {
            zv = dinv[i] * rv;
            zg[i] = zv;
        } else {
            zv = zg[i];
        }
        s += rv * zv;
    }
    s = block_sum(s, red);
    double tot;
    if (last_block_reduce(s, partials + g * part_stride, counters + g, gridDim.x, blockIdx.x, &tot, red) &&
        threadIdx.x == 0) {
        CgState& st = cg[g];
        if (!(tot > 0.0) || !finite_d(tot)) {
            st.status = finite_d(tot) ? COLA_ERR_NOT_SPD : COLA_ERR_NONFINITE;
            st.active = 0;
            atomicSub(&cnt->num_active, 1);
        } else {
            st.beta = tot / st.rho;
            st.rho = tot;
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_probe_accumulate(const double* Z, const double* Q, int64_t n,
                                                               int nprobes, double scale, double* out,
                                                               int accumulate) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        double s = 0.0;
        for (int j = 0; j < nprobes; ++j) s += Z[(int64_t)j * n + i] * Q[(int64_t)j * n + i];
        out[i] = (accumulate ? out[i] : 0.0) + scale * s;
    }
}

// after the last iteration: report ||r||^2 where plain CG keeps it
__global__ void k_pcg_finish(CgState* cg, int nrhs) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < nrhs) cg[g].rho = cg[g].rho_true;
}

unsigned blocks_for(int64_t n, int max_blocks) {
    int64_t b = (n + (int64_t)kThreads * 16 - 1) / ((int64_t)kThreads * 16);
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (unsigned)b;
}

}  // namespace

hipError_t kron_diagonal(const DiagArgs& a, double* out, bool invert, hipStream_t s) {
    hipLaunchKernelGGL(k_kron_diagonal, dim3(blocks_for(a.n, 4096)), dim3(kThreads), 0, s, a, out, invert ? 1 : 0);
    return hipGetLastError();
}

hipError_t trace_shift(const DiagArgs& a, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_trace_shift, dim3(1), dim3(kThreads), 0, s, a, out);
    return hipGetLastError();
}

hipError_t pcg_update(double* x, double* r, const double* p, const double* q, int64_t n, int nrhs, CgState* cg,
                      double* partials, int part_stride, uint32_t* counters, SolveCounters* cnt, int max_blocks,
                      hipStream_t s, ResHist rh) {
    dim3 grid(blocks_for(n, max_blocks < part_stride ? max_blocks : part_stride), nrhs);
    hipLaunchKernelGGL(k_pcg_update, grid, dim3(kThreads), 0, s, x, r, p, q, n, cg, partials, part_stride,
                       counters, cnt, rh);
    return hipGetLastError();
}

hipError_t pcg_precond_dot(const double* r, double* z, const double* dinv, int64_t n, int nrhs, CgState* cg,
                           double* partials, int part_stride, uint32_t* counters, SolveCounters* cnt,
                           int max_blocks, hipStream_t s) {
    dim3 grid(blocks_for(n, max_blocks < part_stride ? max_blocks : part_stride), nrhs);
    hipLaunchKernelGGL(k_pcg_precond_dot, grid, dim3(kThreads), 0, s, r, z, dinv, n, cg, partials, part_stride,
                       counters, cnt);
    return hipGetLastError();
}

hipError_t pcg_finish(CgState* cg, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_finish, dim3((nrhs + 255) / 256), dim3(256), 0, s, cg, nrhs);
    return hipGetLastError();
}

hipError_t probe_accumulate(const double* Z, const double* Q, int64_t n, int nprobes, double scale, double* out,
                            bool accumulate, hipStream_t s) {
    hipLaunchKernelGGL(k_probe_accumulate, dim3(blocks_for(n, 4096)), dim3(kThreads), 0, s, Z, Q, n, nprobes,
                       scale, out, accumulate ? 1 : 0);
    return hipGetLastError();
}

}  // namespace cola
