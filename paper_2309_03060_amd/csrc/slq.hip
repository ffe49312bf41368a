// Gauss quadrature of log over the Lanczos tridiagonals of a batched CG
// (stochastic Lanczos quadrature of log det A).
//
// LogDet(A) = Tr(Log(A)) for a symmetric PSD operator (App. A, derived
// functions), and stochastic Lanczos quadrature is the base-case iterative
// method for such matrix functions (App. C, table of base-case iterative
// algorithms).  For a probe z, k CG iterations on A x = z give the Lanczos
// tridiagonal T_k of the Krylov space of z through the CG-Lanczos relation:
//     T[0][0] = 1 / alpha_0,   T[j][j] = 1 / alpha_j + beta_{j-1} / alpha_{j-1},
//     T[j][j+1] = sqrt(beta_j) / alpha_j,
// and z^T log(A) z ~= ||z||^2 sum_k tau_k^2 log(theta_k), with theta_k the
// eigenvalues of T_k and tau_k the first components of its unit eigenvectors.
// The eigenvalues come from the implicit QL iteration with shifts taken from
// the leading 2 x 2 block; of the accumulated plane rotations only their
// effect on the first row of the eigenvector matrix is kept (tau), so a probe
// costs O(k^2) and three vectors of k doubles, held in LDS.  One thread per
// probe: the probes are independent and k is at most a few thousand.
#include "slq.h"

#include <cmath>

namespace cola {
namespace {

constexpr int kQLSweeps = 64;           // QL iterations per eigenvalue before giving up (NaN)

// ||z||^2 e1^T log(T) e1 for the tridiagonal of k CG iterations with
// coefficients ab[2 j] = alpha_j, ab[2 j + 1] = beta_j; d, e, z: scratch of k.
__device__ double log_quadrature(const double* ab, int k, double znorm2, double* d, double* e, double* z) {
    if (k == 0) return 0.0;                          // z = 0 (no iteration ran)
    d[0] = 1.0 / ab[0];
    for (int j = 1; j < k; ++j) d[j] = 1.0 / ab[2 * j] + ab[2 * j - 1] / ab[2 * j - 2];
    for (int j = 0; j + 1 < k; ++j) e[j] = sqrt(ab[2 * j + 1]) / ab[2 * j];
    e[k - 1] = 0.0;
    for (int j = 0; j < k; ++j) z[j] = j == 0 ? 1.0 : 0.0;
    for (int l = 0; l < k; ++l) {
        int sweeps = 0;
        for (;;) {
            int m = l;                               // the block [l, m] has no negligible coupling
            while (m + 1 < k) {
                const double dd = fabs(d[m]) + fabs(d[m + 1]);
                if (fabs(e[m]) + dd == dd) break;
                ++m;
            }
            if (m == l) break;                       // d[l] has converged
            if (++sweeps > kQLSweeps) return __builtin_nan("");
            // shift: the eigenvalue of the leading 2 x 2 block nearer d[l]
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            bool split = false;
            for (int i = m - 1; i >= l; --i) {       // chase the bulge from the bottom of the block
                const double f = s * e[i], b = c * e[i];
                r = hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {                      // the block splits here: restart on it
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    split = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                const double zt = z[i + 1];          // the rotation acting on the first eigenvector row
                z[i + 1] = s * z[i] + c * zt;
                z[i] = c * z[i] - s * zt;
            }
            if (split) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    double acc = 0.0;
    for (int j = 0; j < k; ++j) acc += z[j] * z[j] * log(d[j]);
    return znorm2 * acc;
}

__global__ void k_slq_probe(const double* hist, int hist_len, const CgState* cg, int nprobes, double* est) {
    extern __shared__ double scratch[];              // 3 hist_len doubles per thread
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nprobes) return;
    double* d = scratch + (size_t)threadIdx.x * 3 * hist_len;
    const CgState& st = cg[g];
    const int k = st.iters < hist_len ? st.iters : hist_len;
    const bool ok = st.status == COLA_OK || st.status == COLA_NOT_CONVERGED;   // a breakdown leaves no quadrature
    est[g] = ok ? log_quadrature(hist + (size_t)g * 2 * hist_len, k, st.bnorm2, d, d + hist_len, d + 2 * hist_len)
                : __builtin_nan("");
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

int slq_threads_per_block(int hist_len) {
    const int t = (int)(kSlqLds / (3 * sizeof(double) * (size_t)hist_len));
    return t < 1 ? 0 : (t > 64 ? 64 : t);
}

hipError_t slq_logdet(const double* hist, int hist_len, const CgState* cg, int nprobes, double* est,
                      double* logdet, hipStream_t s) {
    const int tpb = slq_threads_per_block(hist_len);
    if (tpb < 1 || nprobes < 1) return hipErrorInvalidValue;
    const size_t lds = (size_t)tpb * 3 * hist_len * sizeof(double);
    hipLaunchKernelGGL(k_slq_probe, dim3((unsigned)((nprobes + tpb - 1) / tpb)), dim3(tpb), lds, s, hist, hist_len,
                       cg, nprobes, est);
    hipLaunchKernelGGL(k_slq_mean, dim3(1), dim3(kThreads), 0, s, est, nprobes, logdet);
    return hipGetLastError();
}

}  // namespace cola
