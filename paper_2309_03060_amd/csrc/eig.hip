// Eigendecomposition of Kronecker factors for the Kronecker-eigen solve.
//
// A single Kronecker term K1 (x) .. (x) KF + sigma2 I with symmetric factors
// K_k = Q_k diag(lam_k) Q_k^T has eigenvectors Q1 (x) .. (x) QF and
// eigenvalues lam1 (x) .. (x) lamF + sigma2 (the Kronecker eigenvalue rule of
// the paper's appendix on Kronecker products).  The factors are decomposed
// here with one-sided (Hestenes) Jacobi in FP64: columns of U = A V are
// orthogonalised pairwise by plane rotations accumulated into V.  All n/2
// pairs of one round-robin step are independent, one workgroup each.
#include "eig.h"

#include <algorithm>
#include <cmath>

#include "vector.h"

namespace cola {

namespace {

// Player at table position `pos` in round-robin step `step` (m players, m even):
// player 0 stays, the others rotate, so every pair meets once in m - 1 steps.
__device__ inline int rr_player(int pos, int step, int m) {
    return pos == 0 ? 0 : 1 + (pos - 1 + step) % (m - 1);
}

__global__ __launch_bounds__(kThreads) void k_jacobi_step(double* U, double* V, int64_t n, int m, int step,
                                                          double tol, unsigned long long* off_bits) {
    __shared__ double red[4];
    int p = rr_player(blockIdx.x, step, m);
    int q = rr_player(m - 1 - blockIdx.x, step, m);
    if (p >= n || q >= n) return;                          // the idle player of an odd n
    if (p > q) { const int t = p; p = q; q = t; }
    double* up = U + (int64_t)p * n;
    double* uq = U + (int64_t)q * n;
    double a = 0.0, b = 0.0, g = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kThreads) {
        const double x = up[i], y = uq[i];
        a = __builtin_fma(x, x, a);
        b = __builtin_fma(y, y, b);
        g = __builtin_fma(x, y, g);
    }
    a = block_sum(a, red);
    b = block_sum(b, red);
    g = block_sum(g, red);
    const double ab = sqrt(a * b);
    const double rel = ab > 0.0 ? fabs(g) / ab : 0.0;
    if (threadIdx.x == 0 && rel > 0.0) {
        // non-negative doubles order like their bit patterns
        atomicMax(off_bits, (unsigned long long)__double_as_longlong(rel));
    }
    if (!(rel > tol)) return;
    // rotation that makes columns p and q orthogonal (smaller root of t^2 + 2 zeta t - 1 = 0)
    const double zeta = (b - a) / (2.0 * g);
    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
    double* vp = V + (int64_t)p * n;
    double* vq = V + (int64_t)q * n;
    for (int64_t i = threadIdx.x; i < n; i += kThreads) {
        const double x = up[i], y = uq[i];
        up[i] = c * x - s * y;
        uq[i] = s * x + c * y;
        const double xv = vp[i], yv = vq[i];
        vp[i] = c * xv - s * yv;
        vq[i] = s * xv + c * yv;
    }
}

// U = A (column-major copy of a symmetric matrix), V = I.
__global__ void k_jacobi_init(const double* A, double* U, double* V, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += (int64_t)gridDim.x * blockDim.x) {
        U[e] = A[e];
        V[e] = (e / n == e % n) ? 1.0 : 0.0;
    }
}

// lam_j = v_j . u_j = v_j^T A v_j (the Rayleigh quotient of the converged column).
__global__ __launch_bounds__(kThreads) void k_jacobi_values(const double* U, const double* V, int64_t n, double* lam) {
    __shared__ double red[4];
    const int64_t j = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kThreads) s = __builtin_fma(U[j * n + i], V[j * n + i], s);
    s = block_sum(s, red);
    if (threadIdx.x == 0) lam[j] = s;
}

__global__ void k_transpose_f64(const double* in, double* out, int64_t n) {
    __shared__ double tile[32][33];
    const int64_t bx = (int64_t)blockIdx.x * 32, by = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;        // 256 threads: 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = by + r, j = bx + tx;
        if (i < n && j < n) tile[r][tx] = in[i * n + j];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = bx + r, j = by + tx;
        if (i < n && j < n) out[i * n + j] = tile[tx][r];
    }
}

__global__ void k_eig_scale(const double* Y, double* Z, int64_t total, int64_t n, int64_t n2, int64_t n3,
                            const double* l1, const double* l2, const double* l3, double sigma2) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t rest = e % n;
        const int64_t i3 = rest % n3, i2 = (rest / n3) % n2, i1 = rest / (n2 * n3);
        double lam = l1[i1] * l2[i2];
        if (l3) lam *= l3[i3];
        Z[e] = Y[e] / (lam + sigma2);
    }
}

}  // namespace

int32_t jacobi_eig(const double* A, int64_t n, double* V, double* lam, double* work, double* off, double tol,
                   int max_sweeps, hipStream_t s) {
    if (n < 1 || n > (1 << 20)) return COLA_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_jacobi_init, dim3((unsigned)std::min<int64_t>((n * n + 255) / 256, 65536)), dim3(256), 0,
                       s, A, work, V, n);
    if (hipGetLastError() != hipSuccess) return COLA_ERR_HIP;
    const int m = (int)(n + (n & 1));                      // even number of players
    unsigned long long* bits = (unsigned long long*)off;
    for (int sweep = 0; sweep < max_sweeps && n > 1; ++sweep) {
        if (fill_f64(off, 0.0, 1, s) != hipSuccess) return COLA_ERR_HIP;
        for (int step = 0; step < m - 1; ++step)
            hipLaunchKernelGGL(k_jacobi_step, dim3((unsigned)(m / 2)), dim3(kThreads), 0, s, work, V, n, m, step,
                               tol, bits);
        if (hipGetLastError() != hipSuccess) return COLA_ERR_HIP;
        double h = 0.0;
        if (hipMemcpyAsync(&h, off, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return COLA_ERR_HIP;
        if (!std::isfinite(h)) return COLA_ERR_NONFINITE;
        if (h <= tol) break;
    }
    hipLaunchKernelGGL(k_jacobi_values, dim3((unsigned)n), dim3(kThreads), 0, s, work, V, n, lam);
    return hipGetLastError() == hipSuccess ? COLA_OK : COLA_ERR_HIP;
}

hipError_t eig_scale(const double* Y, double* Z, int64_t nrhs, int F, const int64_t* dims,
                     const double* const* lam, double sigma2, hipStream_t s) {
    int64_t d[3] = {1, 1, 1};
    for (int k = 0; k < F; ++k) d[k] = dims[k];
    const int64_t n = d[0] * d[1] * d[2];
    const int64_t total = nrhs * n;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536));
    hipLaunchKernelGGL(k_eig_scale, dim3(grid), dim3(256), 0, s, Y, Z, total, n, d[1], d[2], lam[0], lam[1],
                       F == 3 ? lam[2] : nullptr, sigma2);
    return hipGetLastError();
}

hipError_t transpose_f64(const double* in, double* out, int64_t n, hipStream_t s) {
    const unsigned g = (unsigned)((n + 31) / 32);
    hipLaunchKernelGGL(k_transpose_f64, dim3(g, g), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}

}  // namespace cola
