// One-workgroup FP64 CG for small two-mode systems.
//
// A system K1 (x) K2 + diag(d) + sigma2 I with modes of at most 64 points has
// n <= 4096 unknowns: its factors, the direction P and the intermediate
// T = P K2^T (the mode-2 product of the per-mode Kronecker MVM, Table 2) fit
// the LDS of one CU, so a whole CG solve runs inside one workgroup with no
// kernel boundary per iteration (a multi-kernel iteration of such a system is
// bound by launch latency, not by its 1 MFLOP).  Both mode products run on the
// FP64 matrix cores (16 x 16 x 4 MFMA): wave w computes output tile
// (w / 4, w % 4) of the 64 x 64 grid, and each thread keeps x, r and p of the
// four elements its MFMA accumulator holds in registers.  Per iteration:
//   T[i][j] = sum_k P[i][k] K2[j][k],   q[i][j] = sum_k K1[i][k] T[k][j] + (sigma2 + d) p
// then the textbook CG step with FP64 block sums in a fixed order.  Padding
// rows and columns hold zeros in P and the factors, so they stay zero.  The
// LDS pitches keep every MFMA operand read free of bank conflicts (one double
// per lane per operand: a tenth of the LDS traffic per multiply-add of plain
// FMAs fed by broadcast reads).
#include "small.h"

namespace cola {
namespace {

constexpr int kST = 1024;               // 16 waves: wave w owns output tile (w / 4, w % 4) of 16 x 16
constexpr int SM = kSmallMax;
constexpr int PA = SM + 2;              // pitch of A operands (P, K1): a half-wave reads 16 rows x 2 columns
constexpr int PB = SM + 16;             // pitch of B operands (K2^T, T): a half-wave reads 2 rows x 16 columns

// Block sum with a single barrier.  The caller alternates between two slot
// arrays (p.q in one, r.r in the other): between the reads of one array and
// its next write every thread passes at least one other barrier of the
// iteration, so no barrier is needed to protect the slots.
__device__ inline double block_sum_small(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kST / 64; ++i) s += red[i];
    return s;
}

__device__ inline doublex4 mma64(double a, double b, doublex4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(kST) void k_small_cg64(SmallArgs a) {
    __shared__ double K1s[SM * PA];     // K1[i][k]
    __shared__ double K2T[SM * PB];     // K2T[k][j] = K2[j][k]
    __shared__ double Ps[SM * PA];      // P[i][k]
    __shared__ double Ts[SM * PB];      // T[k][j] = (P K2^T)[k][j]
    __shared__ double red_rr[kST / 64];    // slots of the b.b and r.r sums
    __shared__ double red_pq[kST / 64];    // slots of the p.q sums
    const int item = blockIdx.x;
    const ResSys sy = a.sys[item / a.nrhs];
    const int rhs = item % a.nrhs;
    const int n1 = sy.n1, n2 = sy.n2;
    const int k1max = (n1 + 15) & ~15, k2max = (n2 + 15) & ~15;  // four MFMA steps of depth 4 at a time;
                                                                   // rows beyond n hold zeros
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int ti = wave >> 2, tj = wave & 3, lr = lane & 15, lk = lane >> 4;
    const int64_t base = (int64_t)a.nrhs * sy.vec_off + (int64_t)rhs * sy.n;
    const double* K1 = a.fac64 + sy.k1_off;
    const double* K2 = a.fac64 + sy.k2_off;
    for (int e = tid; e < SM * SM; e += kST) {
        const int r = e / SM, c = e % SM;
        K1s[r * PA + c] = (r < n1 && c < n1) ? K1[r * n1 + c] : 0.0;
        K2T[r * PB + c] = (r < n2 && c < n2) ? K2[c * n2 + r] : 0.0;
    }
    for (int e = tid; e < SM * PA; e += kST) Ps[e] = 0.0;
    __syncthreads();                                         // factors staged before the first product

    // this thread's elements: the MFMA output layout of tile (ti, tj), element v at
    // row 16 ti + 4 v + lane / 16, column 16 tj + lane % 16
    const int j = 16 * tj + lr;
    // q = A v for this thread's four elements of v: both mode products on the matrix cores
    // through LDS (every thread calls it; its barriers also separate the block sums around it)
    auto apply = [&](const double (&v4)[4], const double (&dd)[4], double (&q)[4]) {
#pragma unroll
        for (int v = 0; v < 4; ++v) Ps[(16 * ti + 4 * v + lk) * PA + j] = v4[v];
        __syncthreads();                                     // P complete
        doublex4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int kb = 0; kb < k2max; kb += 16) {             // T = P K2^T
            double av[4], bv[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                av[s] = Ps[(16 * ti + lr) * PA + kb + 4 * s + lk];
                bv[s] = K2T[(kb + 4 * s + lk) * PB + j];
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) acc = mma64(av[s], bv[s], acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) Ts[(16 * ti + 4 * v + lk) * PB + j] = acc[v];
        __syncthreads();                                     // T complete
        acc = doublex4{0.0, 0.0, 0.0, 0.0};
        for (int kb = 0; kb < k1max; kb += 16) {             // K1 T
            double av[4], bv[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                av[s] = K1s[(16 * ti + lr) * PA + kb + 4 * s + lk];
                bv[s] = Ts[(kb + 4 * s + lk) * PB + j];
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) acc = mma64(av[s], bv[s], acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) q[v] = fma(dd[v], v4[v], acc[v]);
    };
    double x[4], r[4], p[4], dd[4], bvals[4], q[4];
    double bb = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = 16 * ti + 4 * v + lk;
        const bool own = i < n1 && j < n2;
        const int64_t e = (int64_t)i * n2 + j;
        bvals[v] = own ? a.B[base + e] : 0.0;
        x[v] = (own && a.x0_given) ? a.X[base + e] : 0.0;
        dd[v] = own ? sy.sigma2 + (sy.diag_off >= 0 ? a.diag64[sy.diag_off + e] : 0.0) : 0.0;
        bb += bvals[v] * bvals[v];
    }
    bb = block_sum_small(bb, red_rr);
    double rho = bb;
    if (a.x0_given) {                                        // warm start: r0 = b - A x0
        apply(x, dd, q);
        double rr = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            r[v] = bvals[v] - q[v];
            rr += r[v] * r[v];
        }
        rho = block_sum_small(rr, red_pq);
    } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) r[v] = bvals[v];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) p[v] = r[v];
    const double tol2 = a.tol * a.tol * bb;
    int iters = 0, status = COLA_NOT_CONVERGED;
    if (!__builtin_isfinite(bb) || !__builtin_isfinite(rho)) status = COLA_ERR_NONFINITE;
    else if (rho <= tol2) status = COLA_OK;                  // includes b = 0 (x = 0) after zero iterations
    while (status == COLA_NOT_CONVERGED && iters < a.max_iters) {
        apply(p, dd, q);
        double pq = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) pq += p[v] * q[v];
        pq = block_sum_small(pq, red_pq);
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
        rr = block_sum_small(rr, red_rr);
        ++iters;
        const double beta = rr / rho;
        rho = rr;
        if (a.rh.data && tid == 0 && iters % a.rh.stride == 0 && iters / a.rh.stride <= a.rh.len)
            a.rh.data[(int64_t)item * a.rh.len + iters / a.rh.stride - 1] = bb > 0.0 ? sqrt(rr / bb) : sqrt(rr);
        if (!__builtin_isfinite(rr)) status = COLA_ERR_NONFINITE;
        else if (rr <= tol2) status = COLA_OK;
#pragma unroll
        for (int v = 0; v < 4; ++v) p[v] = fma(beta, p[v], r[v]);
    }
    // the FP64 true residual of the returned x
    apply(x, dd, q);
    double rt = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const double e = bvals[v] - q[v];
        rt += e * e;
    }
    rt = block_sum_small(rt, red_pq);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = 16 * ti + 4 * v + lk;
        if (i < n1 && j < n2) a.X[base + (int64_t)i * n2 + j] = x[v];
    }
    if (a.info && tid == 0) {
        cola_solve_info o;
        o.status = status;
        o.iters = iters;
        o.sweeps = 0;
        o.reserved = 0;
        o.relres_recursive = bb > 0.0 ? sqrt(rho / bb) : sqrt(rho);
        o.relres_true = bb > 0.0 ? sqrt(rt / bb) : sqrt(rt);
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
