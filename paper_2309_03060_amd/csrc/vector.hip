// Vector phase of conjugate gradients and of iterative refinement.
//
// CG (the PSD base case of CoLA's solve, Sec. 3.2 / App. C) advances, per
// right-hand side:  x += alpha p,  r -= alpha q,  rho' = r.r,  beta = rho'/rho.
// These kernels stream the vectors once with wide coalesced accesses, keep
// the scalars and every dot-product accumulation in FP64, and reduce the
// per-block partials with the last-block pattern (no second launch, no
// waiting between blocks).  Grids are (blocks per RHS, nrhs): a block never
// straddles two right-hand sides, so converged ones are skipped whole.
#include "vector.h"

namespace cola {

__device__ inline float  fmat(float a, float b, float c)    { return __builtin_fmaf(a, b, c); }
__device__ inline double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T> struct Vec4;
template <> struct Vec4<float>  { using type = floatx4;  static constexpr int W = 4; };
template <> struct Vec4<double> { typedef double __attribute__((ext_vector_type(2))) type; static constexpr int W = 2; };

// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <typename T>
__global__ void k_fill(T* p, T v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_copy_f64(const double* in, double* out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}

// ---------------------------------------------------------------------------
// Refinement setup: ||b||^2 per RHS, x = 0, refinement state.
__global__ __launch_bounds__(kThreads) void k_outer_init(const double* B, double* X, int64_t n,
                                                         OuterState* outer, double tol, int max_sweeps,
                                                         double* partials, int part_stride,
                                                         uint32_t* counters, SolveCounters* cnt, int keep_x) {
    __shared__ double red[4];
    const int64_t g = blockIdx.y;
    const double* b = B + g * n;
    double* x = X + g * n;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const double v = b[i];
        s += v * v;
        if (!keep_x) x[i] = 0.0;
    }
    s = block_sum(s, red);
    double tot;
    if (last_block_reduce(s, partials + g * part_stride, counters + g, gridDim.x, blockIdx.x, &tot, red) &&
        threadIdx.x == 0) {
        OuterState& o = outer[g];
        o.bnorm2 = tot;
        o.rnorm = sqrt(tot);
        o.prev_rnorm = __builtin_inf();
        o.relres = tot > 0.0 ? 1.0 : 0.0;
        o.tol = tol;
        o.slow = 0;
        o.sweeps = 0;
        o.iters = 0;
        o.max_sweeps = max_sweeps;
        if (!finite_d(tot)) {
            o.status = COLA_ERR_NONFINITE;
            o.active = 0;
        } else {
            o.status = COLA_OK;
            o.active = 1;
            atomicAdd(&cnt->num_outer_active, 1);
        }
    }
}

// ---------------------------------------------------------------------------
// Start a CG solve on rhs = src * scale (scale = 1 / ||r|| of the refinement
// residual, or 1): r = rhs, x = 0, p = 0 (so the first direction r + 0 p = r),
// rho = ||r||^2, stop threshold tol^2 ||rhs||^2.
// keep_x: leave x as it is (a warm start, x = x0 with src = b - A x0);
// keep_bnorm: cg.bnorm2 already holds ||b||^2 (tolerances stay relative to b, not to src).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cg_prepare(const double* src, T* r, T* x, T* p, int64_t n,
                                                         const OuterState* outer, CgState* cg, double tol,
                                                         int max_iters, double delta, double* partials,
                                                         int part_stride, uint32_t* counters, SolveCounters* cnt,
                                                         int keep_x, int keep_bnorm) {
    __shared__ double red[4];
    const int64_t g = blockIdx.y;
    if (outer && !outer[g].active) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            cg[g].active = 0;
            cg[g].iters = 0;
            cg[g].status = COLA_OK;
        }
        return;
    }
    const double scale = outer ? 1.0 / outer[g].rnorm : 1.0;
    const double* sg = src + g * n;
    T* rg = r + g * n;
    T* xg = x + g * n;
    T* pg = p + g * n;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const T v = (T)(sg[i] * scale);
        rg[i] = v;
        if (!keep_x) xg[i] = (T)0;
        pg[i] = (T)0;
        s += (double)v * (double)v;
    }
    s = block_sum(s, red);
    double tot;
    if (last_block_reduce(s, partials + g * part_stride, counters + g, gridDim.x, blockIdx.x, &tot, red) &&
        threadIdx.x == 0) {
        CgState& st = cg[g];
        st.rho = tot;
        if (!keep_bnorm) st.bnorm2 = tot;
        st.tol2 = tol * tol * st.bnorm2;
        st.alpha = 0.0;
        st.beta = 0.0;
        st.iters = 0;
        st.max_iters = max_iters;
        st.delta = delta < 0.0 ? -delta : delta;
        st.restart_dir = delta < 0.0;          // a negative delta asks for direction restarts
        st.rmax = sqrt(tot);
        st.rho_true = tot;
        st.need_update = 0;
        st.fails = 0;
        st.updates = 0;
        st.xdefer = 0;
        st.xlag = 0;
        st.pbuf = 0;
        st.pswap = 0;
        if (!finite_d(tot)) {
            st.status = COLA_ERR_NONFINITE;
            st.active = 0;
        } else if (tot <= st.tol2) {      // includes rhs = 0: x = 0 after zero iterations
            st.status = COLA_OK;
            st.active = 0;
        } else {
            st.status = COLA_NOT_CONVERGED;
            st.active = 1;
            atomicAdd(&cnt->num_active, 1);
        }
    }
}

// cg.bnorm2 = ||b||^2 per right-hand side (the reference of a warm-started solve's tolerance).
__global__ __launch_bounds__(kThreads) void k_rhs_norm2(const double* B, int64_t n, CgState* cg, double* partials,
                                                        int part_stride, uint32_t* counters) {
    __shared__ double red[4];
    const int64_t g = blockIdx.y;
    const double* bg = B + g * n;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        s += bg[i] * bg[i];
    s = block_sum(s, red);
    double tot;
    if (last_block_reduce(s, partials + g * part_stride, counters + g, gridDim.x, blockIdx.x, &tot, red) &&
        threadIdx.x == 0)
        cg[g].bnorm2 = tot;
}

// ---------------------------------------------------------------------------
// x += alpha p;  r -= alpha q;  rho' = r.r (FP64);  last block: convergence test and beta.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cg_update(T* x, T* r, const T* p, const T* q, int64_t n,
                                                        CgState* cg, double* partials, int part_stride,
                                                        uint32_t* counters, SolveCounters* cnt, double* hist,
                                                        int hist_len, ResHist rh, int streaming) {
    __shared__ double red[4];
    const int64_t g = blockIdx.y;
    if (!cg[g].active) return;
    const T alpha = (T)cg[g].alpha;
    T* xg = x + g * n;
    T* rg = r + g * n;
    const T* pg = p + g * n;
    const T* qg = q + g * n;
    double s = 0.0;
    using VT = typename Vec4<T>::type;
    constexpr int W = Vec4<T>::W;
    const int64_t nv = (n % W == 0) ? n / W : 0;      // vector path when rows stay aligned
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    const bool defer = cg[g].xdefer != 0;               // x += alpha p left to the next first pass
    if (defer) {
        for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nv; i += stride) {
            VT rv = ((VT*)rg)[i];
            const VT qv = ((const VT*)qg)[i];
#pragma unroll
            for (int c = 0; c < W; ++c) {
                rv[c] = fmat(-alpha, qv[c], rv[c]);
                s += (double)rv[c] * (double)rv[c];
            }
            ((VT*)rg)[i] = rv;
        }
    }
    if (streaming) {                                    // working set beyond the last-level cache
        for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; !defer && i < nv; i += stride) {
            VT xv = __builtin_nontemporal_load((VT*)xg + i), rv = __builtin_nontemporal_load((VT*)rg + i);
            const VT pv = __builtin_nontemporal_load((const VT*)pg + i);
            const VT qv = __builtin_nontemporal_load((const VT*)qg + i);
#pragma unroll
            for (int c = 0; c < W; ++c) {
                xv[c] = fmat(alpha, pv[c], xv[c]);
                rv[c] = fmat(-alpha, qv[c], rv[c]);
                s += (double)rv[c] * (double)rv[c];
            }
            __builtin_nontemporal_store(xv, (VT*)xg + i);
            __builtin_nontemporal_store(rv, (VT*)rg + i);
        }
    }
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; !streaming && !defer && i < nv; i += stride) {
        VT xv = ((VT*)xg)[i], rv = ((VT*)rg)[i];
        const VT pv = ((const VT*)pg)[i], qv = ((const VT*)qg)[i];
#pragma unroll
        for (int c = 0; c < W; ++c) {
            xv[c] = fmat(alpha, pv[c], xv[c]);
            rv[c] = fmat(-alpha, qv[c], rv[c]);
            s += (double)rv[c] * (double)rv[c];
        }
        ((VT*)xg)[i] = xv;
        ((VT*)rg)[i] = rv;
    }
    for (int64_t i = nv * W + (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        const T rv = fmat(-alpha, qg[i], rg[i]);
        if (!defer) xg[i] = fmat(alpha, pg[i], xg[i]);
        rg[i] = rv;
        s += (double)rv * (double)rv;
    }
    s = block_sum(s, red);
    double tot;
    if (last_block_reduce(s, partials + g * part_stride, counters + g, gridDim.x, blockIdx.x, &tot, red) &&
        threadIdx.x == 0) {
        CgState& st = cg[g];
        st.iters += 1;
        if (st.xdefer) st.xlag = 1;                      // x now lacks alpha p of this step
        if (st.pswap) st.pbuf ^= 1;                      // this step's direction is in the other buffer
        if (hist && st.iters <= hist_len) {      // the CG coefficients behind the Lanczos tridiagonal
            double* h = hist + ((int64_t)g * hist_len + st.iters - 1) * 2;
            h[0] = st.alpha;
            h[1] = tot / st.rho;
        }
        record_residual(rh, g, st, tot);
        bool stop = true;
        if (!finite_d(tot)) {
            st.status = COLA_ERR_NONFINITE;
        } else if (tot <= st.tol2) {
            // plain CG: converged.  Reliable updates: pause and let the FP64
            // residual at the end of the chunk decide.
            if (st.delta > 0.0) st.need_update = 1;
            else st.status = COLA_OK;
        } else if (st.iters >= st.max_iters) {
            st.status = COLA_NOT_CONVERGED;
        } else {
            stop = false;
            if (st.delta > 0.0 && tot < st.delta * st.delta * st.rmax * st.rmax) {
                st.need_update = 1;
                if (tot < kNoiseFloor * kNoiseFloor * st.rmax * st.rmax) {
                    st.need_update = kNoisePause;
                    stop = true;
                }
            }
        }
        st.beta = tot / st.rho;
        st.rho = tot;
        if (stop) {
            st.active = 0;
            atomicSub(&cnt->num_active, 1);
        }
    }
}

// ---------------------------------------------------------------------------
// x64 += ||r|| * d  for every RHS that ran an inner solve this sweep.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_refine_accumulate(double* x64, const T* d, int64_t n,
                                                                const OuterState* outer) {
    const int64_t g = blockIdx.y;
    if (!outer[g].active) return;
    const double c = outer[g].rnorm;
    double* xg = x64 + g * n;
    const T* dg = d + g * n;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        xg[i] = __builtin_fma(c, (double)dg[i], xg[i]);
}

// Sweep bookkeeping (one thread per RHS): count the sweep and its inner
// iterations; an inner breakdown ends refinement for that RHS.
__global__ void k_outer_bookkeep(OuterState* outer, const CgState* cg, int nrhs, SolveCounters* cnt) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nrhs) return;
    OuterState& o = outer[g];
    if (!o.active) return;
    o.sweeps += 1;
    o.iters += cg[g].iters;
    const int st = cg[g].status;
    if (st == COLA_ERR_NOT_SPD || st == COLA_ERR_NONFINITE) {
        o.status = st;
        o.active = 0;
        atomicSub(&cnt->num_outer_active, 1);
    }
}

// Reliable update, step 1 (gated on need_update, or every RHS when
// all_rhs): fold the low-precision iterate into the FP64 solution, x_lo = 0.
// An iterate whose last step is still deferred (xlag) gets alpha p first, in
// the working precision, as the vector update would have applied it (p from
// the second direction buffer p2 when pbuf says so).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_reliable_fold(double* x64, T* xlo, const T* p, const T* p2, int64_t n,
                                                            const CgState* cg, int all_rhs) {
    const int64_t g = blockIdx.y;
    if (!all_rhs && !cg[g].need_update) return;
    double* xg = x64 + g * n;
    T* lg = xlo + g * n;
    const bool lag = p && cg[g].xlag;
    const T alpha = (T)cg[g].alpha;
    const T* pb = (p2 && cg[g].pbuf) ? p2 : p;
    const T* pg = pb ? pb + g * n : nullptr;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const T v = lag ? fmat(alpha, pg[i], lg[i]) : lg[i];
        xg[i] += (double)v;
        lg[i] = (T)0;
    }
}

// Reliable update, step 3 (after the FP64 residual r64 = b - A x64 and its
// norm rho_true): r_lo = r64; the last block decides convergence from the
// true residual, resumes a paused RHS, and rescales beta so the next
// direction is r_new + (rho_true / rho_old) p.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_reliable_apply(const double* r64, T* rlo, int64_t n, CgState* cg,
                                                             double* partials, int part_stride, uint32_t* counters,
                                                             SolveCounters* cnt) {
    __shared__ double red[4];
    const int64_t g = blockIdx.y;
    if (!cg[g].need_update) return;
    const double* rg = r64 + g * n;
    T* lg = rlo + g * n;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
        lg[i] = (T)rg[i];
    double tot;
    if (last_block_reduce(0.0, partials + g * part_stride, counters + g, gridDim.x, blockIdx.x, &tot, red) &&
        threadIdx.x == 0) {
        cg[g].xlag = 0;                                  // the fold applied any deferred step
        reliable_finish(cg[g], cnt);
    }
}

// Public per-RHS outcome: the recursive residual of the (inner) CG and the FP64
// true residual of the returned x.
__global__ void k_write_info(cola_solve_info* info, const OuterState* outer, const CgState* cg, int nrhs) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nrhs) return;
    cola_solve_info o;
    if (outer) {                                 // restarted refinement: its test is on the true residual
        o.status = outer[g].status;
        o.iters = outer[g].iters;
        o.sweeps = outer[g].sweeps;
        o.relres_recursive = outer[g].relres;
        o.relres_true = outer[g].relres;
    } else {
        const CgState& st = cg[g];
        const double b2 = st.bnorm2;
        o.status = st.status;
        o.iters = st.iters;
        o.sweeps = st.delta > 0.0 ? st.updates : 0;
        o.relres_recursive = b2 > 0.0 ? sqrt(st.rho / b2) : sqrt(st.rho);
        o.relres_true = b2 > 0.0 ? sqrt(st.rho_true / b2) : sqrt(st.rho_true);
        // reliable updates stop on the true residual
        if (st.delta > 0.0 && o.status == COLA_NOT_CONVERGED && b2 > 0.0 && st.rho_true <= st.tol2) o.status = COLA_OK;
    }
    o.reserved = 0;
    info[g] = o;
}

// need_update = 1 exactly for the right-hand sides that did not finish with a
// certified true residual (used by the final fold of a reliable-update solve).
__global__ void k_mark_unverified(CgState* cg, int nrhs) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < nrhs) cg[g].need_update = cg[g].status != COLA_OK ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Factor / vector conversions (round to nearest even at every narrowing).
__global__ void k_f64_to_f32(const double* in, float* out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
}
__global__ void k_f32_to_f64(const float* in, double* out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (double)in[i];
}
// bf16 split: parts[s] = bf16(remainder after the previous parts), remainder kept in FP32.
__global__ void k_f64_to_bf16_split(const double* in, __bf16* out, int64_t n, int nparts, int64_t plane) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float rest = (float)in[i];
        for (int s = 0; s < nparts; ++s) {
            const __bf16 h = (__bf16)rest;
            out[s * plane + i] = h;
            rest = rest - (float)h;
        }
    }
}

// ---------------------------------------------------------------------------
static inline unsigned grid_for(int64_t n, int64_t per_block, int64_t cap) {
    int64_t b = (n + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

int vec_blocks_per_rhs(int64_t n) {
    // about 16 elements per thread, at most 512 blocks per RHS
    return (int)grid_for(n, (int64_t)kThreads * 16, 512);
}

hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256, 1 << 20)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t fill_f64(double* p, double v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n, 256 * 8, 65536)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}
hipError_t copy_f64(const double* in, double* out, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_f64, dim3(grid_for(n, 256 * 8, 65536)), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}
hipError_t fill_f32(float* p, float v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(n, 256 * 8, 65536)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t outer_init(const double* B, double* X, int64_t n, int nrhs, OuterState* outer, double tol,
                      int max_sweeps, double* partials, int part_stride, uint32_t* counters,
                      SolveCounters* cnt, hipStream_t s, bool keep_x) {
    dim3 grid(vec_blocks_per_rhs(n), nrhs);
    hipLaunchKernelGGL(k_outer_init, grid, dim3(kThreads), 0, s, B, X, n, outer, tol, max_sweeps,
                       partials, part_stride, counters, cnt, keep_x ? 1 : 0);
    return hipGetLastError();
}

template <typename T>
hipError_t cg_prepare(const double* src, T* r, T* x, T* p, int64_t n, int nrhs, const OuterState* outer,
                      CgState* cg, double tol, int max_iters, double delta, double* partials, int part_stride,
                      uint32_t* counters, SolveCounters* cnt, hipStream_t s, bool keep_x, bool keep_bnorm) {
    dim3 grid(vec_blocks_per_rhs(n), nrhs);
    hipLaunchKernelGGL(k_cg_prepare<T>, grid, dim3(kThreads), 0, s, src, r, x, p, n, outer, cg, tol,
                       max_iters, delta, partials, part_stride, counters, cnt, keep_x ? 1 : 0, keep_bnorm ? 1 : 0);
    return hipGetLastError();
}
template hipError_t cg_prepare<float>(const double*, float*, float*, float*, int64_t, int, const OuterState*,
                                      CgState*, double, int, double, double*, int, uint32_t*, SolveCounters*,
                                      hipStream_t, bool, bool);
template hipError_t cg_prepare<double>(const double*, double*, double*, double*, int64_t, int, const OuterState*,
                                       CgState*, double, int, double, double*, int, uint32_t*, SolveCounters*,
                                       hipStream_t, bool, bool);

hipError_t rhs_norm2(const double* B, int64_t n, int nrhs, CgState* cg, double* partials, int part_stride,
                     uint32_t* counters, hipStream_t s) {
    dim3 grid(vec_blocks_per_rhs(n), nrhs);
    hipLaunchKernelGGL(k_rhs_norm2, grid, dim3(kThreads), 0, s, B, n, cg, partials, part_stride, counters);
    return hipGetLastError();
}

template <typename T>
hipError_t reliable_fold(double* x64, T* xlo, const T* p, const T* p2, int64_t n, int nrhs, const CgState* cg,
                         bool all_rhs, hipStream_t s) {
    dim3 grid(vec_blocks_per_rhs(n), nrhs);
    hipLaunchKernelGGL(k_reliable_fold<T>, grid, dim3(kThreads), 0, s, x64, xlo, p, p2, n, cg, all_rhs ? 1 : 0);
    return hipGetLastError();
}
template hipError_t reliable_fold<float>(double*, float*, const float*, const float*, int64_t, int, const CgState*,
                                         bool, hipStream_t);

template <typename T>
hipError_t reliable_apply(const double* r64, T* rlo, int64_t n, int nrhs, CgState* cg, double* partials,
                          int part_stride, uint32_t* counters, SolveCounters* cnt, hipStream_t s) {
    dim3 grid(vec_blocks_per_rhs(n), nrhs);
    hipLaunchKernelGGL(k_reliable_apply<T>, grid, dim3(kThreads), 0, s, r64, rlo, n, cg, partials, part_stride,
                       counters, cnt);
    return hipGetLastError();
}
template hipError_t reliable_apply<float>(const double*, float*, int64_t, int, CgState*, double*, int, uint32_t*,
                                          SolveCounters*, hipStream_t);

template <typename T>
hipError_t cg_update(T* x, T* r, const T* p, const T* q, int64_t n, int nrhs, CgState* cg, double* partials,
                     int part_stride, uint32_t* counters, SolveCounters* cnt, hipStream_t s, double* hist,
                     int hist_len, ResHist rh) {
    dim3 grid(vec_blocks_per_rhs(n), nrhs);
    // the four vectors of every right-hand side at once beyond the 256 MiB last-level cache:
    // nothing of them survives to their next use, so they bypass it (non-temporal accesses)
    const int streaming = 4.0 * (double)n * nrhs * sizeof(T) > 256.0 * (1 << 20) ? 1 : 0;
    hipLaunchKernelGGL(k_cg_update<T>, grid, dim3(kThreads), 0, s, x, r, p, q, n, cg, partials, part_stride,
                       counters, cnt, hist, hist_len, rh, streaming);
    return hipGetLastError();
}
template hipError_t cg_update<float>(float*, float*, const float*, const float*, int64_t, int, CgState*, double*,
                                     int, uint32_t*, SolveCounters*, hipStream_t, double*, int, ResHist);
template hipError_t cg_update<double>(double*, double*, const double*, const double*, int64_t, int, CgState*,
                                      double*, int, uint32_t*, SolveCounters*, hipStream_t, double*, int, ResHist);

template <typename T>
hipError_t refine_accumulate(double* x64, const T* d, int64_t n, int nrhs, const OuterState* outer,
                             hipStream_t s) {
    dim3 grid(vec_blocks_per_rhs(n), nrhs);
    hipLaunchKernelGGL(k_refine_accumulate<T>, grid, dim3(kThreads), 0, s, x64, d, n, outer);
    return hipGetLastError();
}
template hipError_t refine_accumulate<float>(double*, const float*, int64_t, int, const OuterState*, hipStream_t);
template hipError_t refine_accumulate<double>(double*, const double*, int64_t, int, const OuterState*, hipStream_t);

hipError_t outer_bookkeep(OuterState* outer, const CgState* cg, int nrhs, SolveCounters* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_outer_bookkeep, dim3((nrhs + 255) / 256), dim3(256), 0, s, outer, cg, nrhs, cnt);
    return hipGetLastError();
}

hipError_t write_info(cola_solve_info* info, const OuterState* outer, const CgState* cg, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_write_info, dim3((nrhs + 255) / 256), dim3(256), 0, s, info, outer, cg, nrhs);
    return hipGetLastError();
}

hipError_t mark_unverified(CgState* cg, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_mark_unverified, dim3((nrhs + 255) / 256), dim3(256), 0, s, cg, nrhs);
    return hipGetLastError();
}

hipError_t convert_f64_f32(const double* in, float* out, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_f64_to_f32, dim3(grid_for(n, 256 * 4, 65536)), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}
hipError_t convert_f32_f64(const float* in, double* out, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_f32_to_f64, dim3(grid_for(n, 256 * 4, 65536)), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}
hipError_t convert_f64_bf16_split(const double* in, __bf16* out, int64_t n, int nparts, int64_t plane,
                                  hipStream_t s) {
    hipLaunchKernelGGL(k_f64_to_bf16_split, dim3(grid_for(n, 256 * 4, 65536)), dim3(256), 0, s, in, out, n,
                       nparts, plane);
    return hipGetLastError();
}

}  // namespace cola
