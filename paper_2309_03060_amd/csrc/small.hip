// One-workgroup FP64 CG for small two-mode systems.
//
// A system K1 (x) K2 + diag(d) + sigma2 I with modes of at most 64 points has
// n <= 4096 unknowns: its factors, the direction P and the intermediate
// T = P K2^T (the mode-2 product of the per-mode Kronecker MVM, Table 2) fit
// the LDS of one CU, so a whole CG solve runs inside one workgroup with no
// kernel boundary per iteration (a multi-kernel iteration of such a system is
// bound by launch latency, not by its 1 MFLOP).  Wave w owns rows
// 4w .. 4w + 3 of the n1 x n2 grid and lane l column l; each thread keeps its
// four elements of x, r and p in registers.  Per iteration:
//   T[i][j] = sum_k P[i][k] K2[j][k]     (P read transposed: 4 rows per LDS broadcast)
//   q[i][j] = sum_k K1[i][k] T[k][j] + (sigma2 + d) p
// then the textbook CG step with FP64 block sums in a fixed order.  Padding
// rows and columns hold zeros in P and the factors, so they stay zero.
#include "small.h"

namespace cola {
namespace {

constexpr int kST = 1024;               // 16 waves
constexpr int SM = kSmallMax;
constexpr int PS = SM + 1;              // row stride of P^T (odd: spreads the transposed stores over banks)

__device__ inline double block_sum_small(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kST / 64; ++i) s += red[i];
    __syncthreads();
    return s;
}

__global__ __launch_bounds__(kST) void k_small_cg64(SmallArgs a) {
    __shared__ double K1T[SM * SM];     // K1T[k][i] = K1[i][k]
    __shared__ double K2T[SM * SM];     // K2T[k][j] = K2[j][k]
    __shared__ double PT[SM * PS];      // PT[k][i] = P[i][k]
    __shared__ double Ts[SM * SM];      // T[i][j]
    __shared__ double red[kST / 64];
    const int item = blockIdx.x;
    const ResSys sy = a.sys[item / a.nrhs];
    const int rhs = item % a.nrhs;
    const int n1 = sy.n1, n2 = sy.n2;
    const int k1max = (n1 + 7) & ~7, k2max = (n2 + 7) & ~7;   // <= kSmallMax
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t base = (int64_t)a.nrhs * sy.vec_off + (int64_t)rhs * sy.n;
    const double* K1 = a.fac64 + sy.k1_off;
    const double* K2 = a.fac64 + sy.k2_off;
    for (int e = tid; e < SM * SM; e += kST) {
        const int k = e / SM, i = e % SM;
        K1T[e] = (k < n1 && i < n1) ? K1[i * n1 + k] : 0.0;
        K2T[e] = (k < n2 && i < n2) ? K2[i * n2 + k] : 0.0;
    }
    for (int e = tid; e < SM * PS; e += kST) PT[e] = 0.0;

    // this thread's elements: rows 4 wave + v, column lane
    double x[4], r[4], p[4], dd[4];
    double bb = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = 4 * wave + v;
        const bool own = i < n1 && lane < n2;
        const int64_t e = (int64_t)i * n2 + lane;
        r[v] = own ? a.B[base + e] : 0.0;
        x[v] = 0.0;
        p[v] = r[v];
        dd[v] = own ? sy.sigma2 + (sy.diag_off >= 0 ? a.diag64[sy.diag_off + e] : 0.0) : 0.0;
        bb += r[v] * r[v];
    }
    bb = block_sum_small(bb, red);
    const double tol2 = a.tol * a.tol * bb;
    double rho = bb;
    int iters = 0, status = COLA_NOT_CONVERGED;
    if (!__builtin_isfinite(bb)) status = COLA_ERR_NONFINITE;
    else if (bb <= tol2) status = COLA_OK;                  // includes b = 0: x = 0 after zero iterations
    while (status == COLA_NOT_CONVERGED && iters < a.max_iters) {
#pragma unroll
        for (int v = 0; v < 4; ++v) PT[lane * PS + 4 * wave + v] = p[v];
        __syncthreads();                                     // P complete
        // k runs to a multiple of 8: rows k >= n2 of P^T and K2^T hold zeros
        double t[4] = {0.0, 0.0, 0.0, 0.0};
        for (int kb = 0; kb < k2max; kb += 8) {
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                const int k = kb + kk;
                const double kv = K2T[k * SM + lane];
#pragma unroll
                for (int v = 0; v < 4; ++v) t[v] = fma(PT[k * PS + 4 * wave + v], kv, t[v]);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) Ts[(4 * wave + v) * SM + lane] = t[v];
        __syncthreads();                                     // T complete
        // rows k >= n1 of T and K1^T hold zeros (P^T has zero columns there)
        double q[4] = {0.0, 0.0, 0.0, 0.0};
        for (int kb = 0; kb < k1max; kb += 8) {
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                const int k = kb + kk;
                const double tv = Ts[k * SM + lane];
#pragma unroll
                for (int v = 0; v < 4; ++v) q[v] = fma(K1T[k * SM + 4 * wave + v], tv, q[v]);
            }
        }
        double pq = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            q[v] = fma(dd[v], p[v], q[v]);
            pq += p[v] * q[v];
        }
        pq = block_sum_small(pq, red);
        if (!(pq > 0.0) || !__builtin_isfinite(pq)) {
            status = __builtin_isfinite(pq) ? COLA_ERR_NOT_SPD : COLA_ERR_NONFINITE;
            break;
        }
        const double alpha = rho / pq;
        double rr = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            x[v] = fma(alpha, p[v], x[v]);
            r[v] = fma(-alpha, q[v], r[v]);
            rr += r[v] * r[v];
        }
        rr = block_sum_small(rr, red);
        ++iters;
        const double beta = rr / rho;
        rho = rr;
        if (!__builtin_isfinite(rr)) status = COLA_ERR_NONFINITE;
        else if (rr <= tol2) status = COLA_OK;
#pragma unroll
        for (int v = 0; v < 4; ++v) p[v] = fma(beta, p[v], r[v]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = 4 * wave + v;
        if (i < n1 && lane < n2) a.X[base + (int64_t)i * n2 + lane] = x[v];
    }
    if (a.info && tid == 0) {
        cola_solve_info o;
        o.status = status;
        o.iters = iters;
        o.sweeps = 0;
        o.reserved = 0;
        o.relres = bb > 0.0 ? sqrt(rho / bb) : sqrt(rho);
        a.info[item] = o;
    }
}

}  // namespace

hipError_t launch_small_cg64(const SmallArgs& a, hipStream_t s) {
    if (a.nitems < 1) return hipSuccess;
    hipLaunchKernelGGL(k_small_cg64, dim3((unsigned)a.nitems), dim3(kST), 0, s, a);
    return hipGetLastError();
}

}  // namespace cola
