// Gauss quadrature of log over the Lanczos tridiagonals of a batched CG
// (stochastic Lanczos quadrature of log det A).
//
// LogDet(A) = Tr(Log(A)) for a symmetric PSD operator (App. A, derived
// functions), and stochastic Lanczos quadrature is the base-case iterative
// method for such matrix functions (App. C, table of base-case iterative
// algorithms).  For a probe z, k CG iterations on A x = z give the Lanczos
// tridiagonal T_k of the Krylov space of z through the CG-Lanczos relation:
//     T[0][0] = 1 / alpha_0,   T[j][j] = 1 / alpha_j + beta_{j-1} / alpha_{j-1},
//     T[j][j+1]^2 = beta_j / alpha_j^2,
// and z^T log(A) z ~= ||z||^2 e1^T log(T_k) e1, the value of the k-node Gauss
// quadrature rule (eigenvalues of T_k as nodes, squared first eigenvector
// components as weights).
//
// That value is computed here without the eigendecomposition, from the
// integral form of the logarithm of a positive definite matrix:
//     e1^T log(T) e1 = int_0^inf [ 1 / (1 + t) - e1^T (T + t I)^{-1} e1 ] dt,
// where e1^T (T + t I)^{-1} e1 = 1 / g_0(t) with the bottom-up pivots
// g_{k-1} = T[k-1][k-1] + t, g_j = T[j][j] + t - T[j][j+1]^2 / g_{j+1} (all positive
// for t >= 0).  With t = e^u the integrand, a sum of w_j (e^u / (1 + e^u) -
// e^u / (theta_j + e^u)), is analytic in the strip |Im u| < pi and decays
// exponentially in both directions, so the trapezoidal rule in u with step h
// errs by about exp(-2 pi^2 / h) (h = 1/4: 1e-34) once the range covers the
// tails; the tails are bounded from T itself: below the range the integrand is
// about (1 - e1^T T^{-1} e1) t once t is far below the smallest eigenvalue (for
// which 1 / Tr(T^{-1}) is a lower bound within a factor k), above it about
// (T[0][0] - 1) / t^2 once t is far above the largest (Gershgorin bound).  The
// nodes are independent, so a probe is one
// workgroup with every thread on its own nodes: O(nodes * k) work in parallel
// instead of a sequential O(k^2) eigen-iteration per probe.
#include "slq.h"

#include <cmath>

namespace cola {
namespace {

constexpr double kSlqStep = 0.25;       // trapezoidal step in u = log t
constexpr double kSlqTail = 1e-18;      // absolute size of each neglected tail
constexpr int kSlqMaxNodes = 4096;

// e1^T (T + t I)^{-1} e1 by the bottom-up pivots (d: diagonal, o2: squared off-diagonal)
__device__ inline double resolvent_e1(const double* d, const double* o2, int k, double t) {
    double g = d[k - 1] + t;
    for (int j = k - 2; j >= 0; --j) g = d[j] + t - o2[j] / g;
    return 1.0 / g;
}

__global__ __launch_bounds__(kThreads) void k_slq_probe(const double* hist, int hist_len, const CgState* cg,
                                                        int nprobes, double* est) {
    __shared__ double d[kSlqMaxSteps];
    __shared__ double o2[kSlqMaxSteps];
    __shared__ double pf[kSlqMaxSteps];
    __shared__ double red[4];
    __shared__ double s_range[2];
    const int g = blockIdx.x;
    const CgState& st = cg[g];
    const int k = st.iters < hist_len ? st.iters : hist_len;
    const bool ok = st.status == COLA_OK || st.status == COLA_NOT_CONVERGED;   // a breakdown leaves no quadrature
    if (!ok || k == 0) {                                                       // k = 0: zero probe, z^T log(A) z = 0
        if (threadIdx.x == 0) est[g] = ok ? 0.0 : __builtin_nan("");
        return;
    }
    const double* ab = hist + (size_t)g * 2 * hist_len;        // (alpha_j, beta_j) pairs
    for (int j = threadIdx.x; j < k; j += kThreads) {
        const double a = ab[2 * j];
        d[j] = 1.0 / a + (j > 0 ? ab[2 * j - 1] / ab[2 * j - 2] : 0.0);
        o2[j] = j + 1 < k ? ab[2 * j + 1] / (a * a) : 0.0;
    }
    __syncthreads();
    // integration range in u = log t from the tail bounds (one thread, O(k)):
    // forward pivots pf, then backward pivots pb with (T^{-1})[j][j] = 1 / (pf_j + pb_j - d_j)
    if (threadIdx.x == 0) {
        pf[0] = d[0];
        for (int j = 1; j < k; ++j) pf[j] = d[j] - o2[j - 1] / pf[j - 1];
        double pb = d[k - 1], trace = 0.0, gmax = 0.0;
        for (int j = k - 1; j >= 0; --j) {
            if (j < k - 1) pb = d[j] - o2[j] / pb;
            trace += 1.0 / (pf[j] + pb - d[j]);
            const double rad = (j > 0 ? sqrt(o2[j - 1]) : 0.0) + (j + 1 < k ? sqrt(o2[j]) : 0.0);
            gmax = fmax(gmax, d[j] + rad);
        }
        const double f0 = 1.0 / pb;                                     // e1^T T^{-1} e1
        s_range[0] = fmin(log(kSlqTail / fmax(fabs(1.0 - f0), 1e-300)), log(1.0 / trace) - 45.0);
        s_range[1] = log(fmax(fmax(gmax, fabs(d[0] - 1.0)), 1.0) / kSlqTail);
    }
    __syncthreads();
    const double umin = s_range[0], umax = s_range[1];
    int nodes = (int)ceil((umax - umin) / kSlqStep) + 1;
    if (nodes > kSlqMaxNodes) nodes = kSlqMaxNodes;
    double s = 0.0;
    for (int i = threadIdx.x; i < nodes; i += kThreads) {
        const double t = exp(umin + kSlqStep * i);
        s += (1.0 / (1.0 + t) - resolvent_e1(d, o2, k, t)) * t;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) est[g] = st.bnorm2 * kSlqStep * s;
}

// mean over the probes, summed in index order by one block
__global__ __launch_bounds__(kThreads) void k_slq_mean(const double* est, int nprobes, double* out) {
    __shared__ double red[4];
    double s = 0.0;
    for (int g = threadIdx.x; g < nprobes; g += kThreads) s += est[g];
    s = block_sum(s, red);
    if (threadIdx.x == 0) *out = s / nprobes;
}

}  // namespace

hipError_t slq_logdet(const double* hist, int hist_len, const CgState* cg, int nprobes, double* est,
                      double* logdet, hipStream_t s) {
    if (hist_len < 1 || hist_len > kSlqMaxSteps || nprobes < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_slq_probe, dim3((unsigned)nprobes), dim3(kThreads), 0, s, hist, hist_len, cg, nprobes, est);
    hipLaunchKernelGGL(k_slq_mean, dim3(1), dim3(kThreads), 0, s, est, nprobes, logdet);
    return hipGetLastError();
}

}  // namespace cola
