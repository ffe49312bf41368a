// Host-side AddressSanitizer / UndefinedBehaviorSanitizer run of libcola's host code.
//
// Built against a copy of the library whose host code (argument checks, workspace and graph
// caches, tile tables, profiler, every entry point's bookkeeping) is instrumented; the device
// code is built as usual.  Drives every entry point of include/cola.h on small operators through
// the C ABI alone: products (checked against a host product written out from the definition of
// the Kronecker product), FP64, mixed-precision, restarted, preconditioned and warm-started
// solves with residual histories, the adjoint backward, log-determinant and its gradient, the
// diagonal and its estimators, the direct eigen solve, the no-allocation product, autotuning,
// engine switches, profiling and tracing, and the argument errors.  Any sanitizer finding ends
// the process with a report and a non-zero status; so does a failed check.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../include/cola.h"

namespace {

int g_fail = 0;

void check(bool ok, const char* what) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s\n", what);
        g_fail = 1;
    }
}

void ok(int32_t rc, const char* what) {
    if (rc != COLA_OK) {
        std::fprintf(stderr, "FAILED: %s -> %d (%s)\n", what, rc, cola_status_string(rc));
        g_fail = 1;
    }
}

template <typename T>
T* dev_copy(const std::vector<T>& h) {
    T* d = nullptr;
    if (hipMalloc((void**)&d, sizeof(T) * (h.empty() ? 1 : h.size())) != hipSuccess) std::abort();
    if (!h.empty() && hipMemcpy(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice) != hipSuccess)
        std::abort();
    return d;
}

template <typename T>
std::vector<T> host_copy(const T* d, size_t n) {
    std::vector<T> h(n);
    if (hipMemcpy(h.data(), d, sizeof(T) * n, hipMemcpyDeviceToHost) != hipSuccess) std::abort();
    return h;
}

// Symmetric positive definite n x n factor: W W^T / m + shift I (row-major).
std::vector<double> spd(std::mt19937_64& g, int n, double shift) {
    std::normal_distribution<double> N(0.0, 1.0);
    const int m = n + 3;
    std::vector<double> W((size_t)n * m), K((size_t)n * n, 0.0);
    for (double& w : W) w = N(g);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < m; ++k) s += W[(size_t)i * m + k] * W[(size_t)j * m + k];
            K[(size_t)i * n + j] = s / m + (i == j ? shift : 0.0);
        }
    return K;
}

// y = (sum_j U_j (x) V_j + diag(d) + sigma2 I) x for a two-mode system, from the definition
// (A (x) B)[(i, k), (j, l)] = A[i, j] B[k, l] with the row-major vec.
std::vector<double> host_mvm2(const std::vector<std::vector<double>>& U, const std::vector<std::vector<double>>& V,
                              const std::vector<double>& d, double s2, int n1, int n2, const std::vector<double>& x) {
    const size_t n = (size_t)n1 * n2;
    std::vector<double> y(n, 0.0);
    for (size_t t = 0; t < U.size(); ++t)
        for (int i = 0; i < n1; ++i)
            for (int k = 0; k < n2; ++k) {
                double s = 0.0;
                for (int j = 0; j < n1; ++j)
                    for (int l = 0; l < n2; ++l)
                        s += U[t][(size_t)i * n1 + j] * V[t][(size_t)k * n2 + l] * x[(size_t)j * n2 + l];
                y[(size_t)i * n2 + k] += s;
            }
    for (size_t e = 0; e < n; ++e) y[e] += (s2 + (d.empty() ? 0.0 : d[e])) * x[e];
    return y;
}

cola_solve_opts base_opts(int prec) {
    cola_solve_opts o{};
    o.tol = 1e-9;
    o.max_iters = 500;
    o.prec = prec;
    o.inner_tol = 0.1;
    o.max_sweeps = 20;
    o.check_every = 8;
    o.refine = COLA_REFINE_RELIABLE;
    o.precond = COLA_PRECOND_NONE;
    return o;
}

void expect_ok_infos(const cola_solve_info* dinfo, int count, double tol, const char* what) {
    auto info = host_copy(dinfo, (size_t)count);
    for (int i = 0; i < count; ++i) {
        if (info[i].status != COLA_OK || !(info[i].relres_true <= tol)) {
            std::fprintf(stderr, "FAILED: %s rhs %d status %d relres_true %g\n", what, i, info[i].status,
                         info[i].relres_true);
            g_fail = 1;
        }
    }
}

}  // namespace

int main() {
    std::mt19937_64 g(2309);
    std::normal_distribution<double> N(0.0, 1.0);
    cola_trace_enable(1);

    // ---- a two-system op: a sum of two terms with a diagonal, and one term without ----
    const int n1 = 24, n2 = 20, m1 = 16, m2 = 12;
    std::vector<std::vector<double>> U = {spd(g, n1, 0.1), spd(g, n1, 0.1)};
    std::vector<std::vector<double>> V = {spd(g, n2, 0.1), spd(g, n2, 0.1)};
    std::vector<double> dg((size_t)n1 * n2);
    for (double& v : dg) v = 0.5 + 0.5 * std::fabs(N(g));
    std::vector<double> P = spd(g, m1, 0.2), Q = spd(g, m2, 0.2);
    double *dU0 = dev_copy(U[0]), *dU1 = dev_copy(U[1]), *dV0 = dev_copy(V[0]), *dV1 = dev_copy(V[1]);
    double *dP = dev_copy(P), *dQ = dev_copy(Q), *dd = dev_copy(dg);
    const void* f0[4] = {dU0, dV0, dU1, dV1};
    const void* f1[2] = {dP, dQ};
    cola_system_desc sys[2] = {};
    sys[0].nterms = 2; sys[0].nfactors = 2; sys[0].dims[0] = n1; sys[0].dims[1] = n2;
    sys[0].factors = f0; sys[0].diag = dd; sys[0].sigma2 = 0.05;
    sys[1].nterms = 1; sys[1].nfactors = 2; sys[1].dims[0] = m1; sys[1].dims[1] = m2;
    sys[1].factors = f1; sys[1].diag = nullptr; sys[1].sigma2 = 0.3;
    cola_op_t op = nullptr;
    ok(cola_op_create(sys, 2, COLA_PREC_FP32, nullptr, &op), "op_create");
    int64_t ntot = 0;
    int32_t nsys = 0;
    ok(cola_op_size(op, &ntot, &nsys), "op_size");
    check(ntot == (int64_t)n1 * n2 + m1 * m2 && nsys == 2, "op_size values");
    const int nrhs = 3;
    const size_t vn = (size_t)nrhs * ntot;

    // ---- products ----
    std::vector<double> xh(vn), yh_ref(vn);
    for (double& v : xh) v = N(g);
    double* dx = dev_copy(xh);
    double* dy = dev_copy(std::vector<double>(vn, 0.0));
    ok(cola_kron_matvec(op, dx, dy, nrhs, COLA_F64, COLA_PREC_FP64, nullptr), "matvec fp64");
    {
        auto yh = host_copy(dy, vn);
        double err = 0.0, scale = 0.0;
        for (int r = 0; r < nrhs; ++r) {
            std::vector<double> x0(xh.begin() + (size_t)r * n1 * n2, xh.begin() + (size_t)(r + 1) * n1 * n2);
            auto y0 = host_mvm2(U, V, dg, 0.05, n1, n2, x0);
            for (size_t e = 0; e < y0.size(); ++e) {
                err = std::fmax(err, std::fabs(yh[(size_t)r * n1 * n2 + e] - y0[e]));
                scale = std::fmax(scale, std::fabs(y0[e]));
            }
            const size_t off = (size_t)nrhs * n1 * n2 + (size_t)r * m1 * m2;
            std::vector<double> x1(xh.begin() + off, xh.begin() + off + (size_t)m1 * m2);
            auto y1 = host_mvm2({P}, {Q}, {}, 0.3, m1, m2, x1);
            for (size_t e = 0; e < y1.size(); ++e) err = std::fmax(err, std::fabs(yh[off + e] - y1[e]));
        }
        check(err <= 1e-12 * scale, "fp64 product against the host definition");
    }
    std::vector<float> xf(vn);
    for (size_t e = 0; e < vn; ++e) xf[e] = (float)xh[e];
    float* dxf = dev_copy(xf);
    float* dyf = dev_copy(std::vector<float>(vn, 0.f));
    float* dyf2 = dev_copy(std::vector<float>(vn, 0.f));
    ok(cola_kron_matvec(op, dxf, dyf, nrhs, COLA_F32, COLA_PREC_FP32, nullptr), "matvec fp32");
    ok(cola_kron_matvec_noalloc(op, dxf, dyf2, nrhs, COLA_F32, COLA_PREC_FP32, nullptr), "matvec noalloc");
    ok(cola_kron_matvec_noalloc(op, dxf, dyf2, 1, COLA_F32, COLA_PREC_FP32, nullptr), "matvec noalloc smaller");
    {
        const float a = host_copy(dyf, vn)[0], b = host_copy(dyf2, vn)[0];
        check(std::fabs(a - b) <= 1e-5f * std::fabs(a) + 1e-6f, "noalloc first entry equals the product's");
    }

    // ---- solves ----
    std::vector<double> bh(vn);
    for (double& v : bh) v = N(g);
    double* db = dev_copy(bh);
    double* dX = dev_copy(std::vector<double>(vn, 0.0));
    cola_solve_info* dinfo = nullptr;
    if (hipMalloc((void**)&dinfo, sizeof(cola_solve_info) * 2 * 16) != hipSuccess) return 2;
    double* dhist = nullptr;
    const int hlen = 40;
    if (hipMalloc((void**)&dhist, sizeof(double) * 2 * nrhs * hlen) != hipSuccess) return 2;

    cola_solve_opts o = base_opts(COLA_PREC_FP64);
    o.hist = dhist; o.hist_len = hlen; o.hist_stride = 2;
    ok(cola_cg_solve(op, db, dX, nrhs, &o, dinfo, nullptr), "solve fp64 with history");
    expect_ok_infos(dinfo, 2 * nrhs, 2e-9, "solve fp64");
    o = base_opts(COLA_PREC_FP32);
    ok(cola_cg_solve(op, db, dX, nrhs, &o, dinfo, nullptr), "solve fp32 reliable");
    expect_ok_infos(dinfo, 2 * nrhs, 1e-9, "solve fp32 reliable");
    o.max_iters = 5;
    ok(cola_cg_solve(op, db, dX, nrhs, &o, dinfo, nullptr), "solve stopped early");
    o.max_iters = 500;
    o.x0_given = 1;
    ok(cola_cg_solve(op, db, dX, nrhs, &o, dinfo, nullptr), "solve resumed");
    expect_ok_infos(dinfo, 2 * nrhs, 1e-9, "solve resumed");
    o = base_opts(COLA_PREC_FP32);
    o.refine = COLA_REFINE_RESTART; o.inner_tol = 1e-3;
    ok(cola_cg_solve(op, db, dX, nrhs, &o, dinfo, nullptr), "solve restarted");
    expect_ok_infos(dinfo, 2 * nrhs, 1e-9, "solve restarted");
    o = base_opts(COLA_PREC_FP64);
    o.precond = COLA_PRECOND_JACOBI;
    ok(cola_cg_solve(op, db, dX, nrhs, &o, dinfo, nullptr), "solve jacobi");
    expect_ok_infos(dinfo, 2 * nrhs, 2e-9, "solve jacobi");
    o.precond = COLA_PRECOND_KRON_EIG;
    ok(cola_cg_solve(op, db, dX, nrhs, &o, dinfo, nullptr), "solve kron-eig");
    expect_ok_infos(dinfo, 2 * nrhs, 2e-9, "solve kron-eig");
    o = base_opts(COLA_PREC_FP32);
    o.check_every = 0;
    ok(cola_cg_solve(op, db, dX, nrhs, &o, dinfo, nullptr), "solve without host waits");

    // ---- backward and gradients ----
    std::vector<double*> gbuf;
    std::vector<void*> dfac;
    for (int t = 0; t < 2; ++t) {
        gbuf.push_back(dev_copy(std::vector<double>((size_t)n1 * n1)));
        gbuf.push_back(dev_copy(std::vector<double>((size_t)n2 * n2)));
    }
    gbuf.push_back(dev_copy(std::vector<double>((size_t)m1 * m1)));
    gbuf.push_back(dev_copy(std::vector<double>((size_t)m2 * m2)));
    for (double* p : gbuf) dfac.push_back(p);
    double* dgd = dev_copy(std::vector<double>((size_t)n1 * n2));
    void* ddiag[2] = {dgd, nullptr};
    double* ds2 = dev_copy(std::vector<double>(2));
    double* dLam = dev_copy(std::vector<double>(vn));
    o = base_opts(COLA_PREC_FP32);
    ok(cola_cg_solve(op, db, dX, nrhs, &o, dinfo, nullptr), "forward for backward");
    ok(cola_cg_solve_backward(op, dX, db, nrhs, &o, dLam, dfac.data(), ddiag, ds2, dinfo, nullptr), "backward");
    expect_ok_infos(dinfo, 2 * nrhs, 1e-9, "backward");
    std::vector<double> zh(vn);
    for (double& v : zh) v = (N(g) > 0.0) ? 1.0 : -1.0;
    double* dz = dev_copy(zh);
    double* dlogdet = dev_copy(std::vector<double>(2));
    double* dest = dev_copy(std::vector<double>(2 * nrhs));
    ok(cola_slq_logdet(op, dz, nrhs, 1e-10, 400, dX, dlogdet, dest, dinfo, nullptr), "slq logdet");
    o = base_opts(COLA_PREC_FP64);
    o.x0_given = 1;
    ok(cola_logdet_grad(op, dz, nrhs, &o, dX, dfac.data(), ddiag, ds2, dinfo, nullptr), "logdet grad");

    // ---- diagonal and estimators ----
    double* ddiagA = dev_copy(std::vector<double>((size_t)ntot));
    ok(cola_op_diagonal(op, ddiagA, nullptr), "op diagonal");
    ok(cola_diag_estimate(op, dz, nrhs, COLA_DIAG_HUTCHINSON, ddiagA, nullptr), "hutchinson");
    std::vector<double> zd((size_t)nrhs * (2 * n1 * n2 + m1 * m2));
    for (double& v : zd) v = (N(g) > 0.0) ? 1.0 : -1.0;
    double* dzd = dev_copy(zd);
    ok(cola_diag_estimate(op, dzd, nrhs, COLA_DIAG_DOUBLY, ddiagA, nullptr), "doubly stochastic");

    // ---- tuning, engines, profiling ----
    ok(cola_autotune(op, nrhs, nullptr), "autotune");
    {
        int64_t len = 0;
        ok(cola_autotune_export(op, nullptr, 0, &len), "tile table length");
        std::vector<char> text((size_t)len + 1);
        ok(cola_autotune_export(op, text.data(), len + 1, &len), "tile table export");
        ok(cola_autotune_import(op, text.data()), "tile table import");
        check(cola_autotune_export(op, text.data(), 1, &len) == COLA_ERR_INVALID_ARG, "export into a short buffer");
        check(cola_autotune_import(op, "device x 1\n1 2 3\n") == COLA_ERR_INVALID_ARG, "malformed table");
    }
    ok(cola_profile_enable(op, 1), "profile on");
    ok(cola_kron_matvec(op, dxf, dyf, nrhs, COLA_F32, COLA_PREC_FP32, nullptr), "profiled product");
    double ms = 0.0;
    int64_t launches = 0;
    ok(cola_profile_read(op, "contract_last", &ms, &launches), "profile read");
    ok(cola_profile_enable(op, 0), "profile off");
    for (int e = 1; e <= 7; ++e) {
        ok(cola_op_set_engine(op, e, 0), "engine off");
        ok(cola_op_set_engine(op, e, 1), "engine on");
    }
    int64_t live = 0, peak = 0;
    ok(cola_op_memory(op, &live, &peak, 1), "op memory");
    check(live > 0 && peak >= live, "op memory values");

    // ---- argument errors ----
    check(cola_kron_matvec(nullptr, dx, dy, 1, COLA_F64, COLA_PREC_FP64, nullptr) == COLA_ERR_INVALID_ARG,
          "null op");
    check(cola_kron_matvec(op, dx, dy, 0, COLA_F64, COLA_PREC_FP64, nullptr) == COLA_ERR_INVALID_ARG, "nrhs 0");
    o = base_opts(COLA_PREC_FP64);
    o.tol = -1.0;
    check(cola_cg_solve(op, db, dX, nrhs, &o, dinfo, nullptr) == COLA_ERR_INVALID_ARG, "negative tol");
    check(cola_op_set_engine(op, 99, 1) == COLA_ERR_INVALID_ARG, "unknown engine");
    for (int32_t s = -8; s <= 3; ++s) check(cola_status_string(s) != nullptr, "status string");
    ok(cola_op_destroy(op), "op destroy");
    ok(cola_op_destroy(nullptr), "destroy null");

    // ---- a one-term three-mode op: the direct eigen solve ----
    std::vector<double> A1 = spd(g, 10, 0.1), A2 = spd(g, 9, 0.1), A3 = spd(g, 8, 0.1);
    double *dA1 = dev_copy(A1), *dA2 = dev_copy(A2), *dA3 = dev_copy(A3);
    const void* f3[3] = {dA1, dA2, dA3};
    cola_system_desc s3 = {};
    s3.nterms = 1; s3.nfactors = 3; s3.dims[0] = 10; s3.dims[1] = 9; s3.dims[2] = 8;
    s3.factors = f3; s3.sigma2 = 0.2;
    cola_op_t op3 = nullptr;
    ok(cola_op_create(&s3, 1, COLA_PREC_BF16X3, nullptr, &op3), "op3 create");
    std::vector<double> b3(720);
    for (double& v : b3) v = N(g);
    double* db3 = dev_copy(b3);
    double* dx3 = dev_copy(std::vector<double>(720));
    ok(cola_eig_solve(op3, db3, dx3, 1, nullptr), "eig solve");
    o = base_opts(COLA_PREC_BF16X3);
    ok(cola_cg_solve(op3, db3, dx3, 1, &o, dinfo, nullptr), "bf16x3 solve");
    expect_ok_infos(dinfo, 1, 1e-9, "bf16x3 solve");
    ok(cola_op_destroy(op3), "op3 destroy");

    for (void* p : {(void*)dU0, (void*)dU1, (void*)dV0, (void*)dV1, (void*)dP, (void*)dQ, (void*)dd, (void*)dx,
                    (void*)dy, (void*)dxf, (void*)dyf, (void*)dyf2, (void*)db, (void*)dX, (void*)dinfo,
                    (void*)dhist, (void*)dgd, (void*)ds2, (void*)dLam, (void*)dz, (void*)dlogdet, (void*)dest,
                    (void*)ddiagA, (void*)dzd, (void*)dA1, (void*)dA2, (void*)dA3, (void*)db3, (void*)dx3})
        (void)hipFree(p);
    for (double* p : gbuf) (void)hipFree(p);
    cola_trace_enable(0);
    std::printf(g_fail ? "host sanitizer run: checks FAILED\n" : "host sanitizer run: all checks passed\n");
    return g_fail;
}
