// Internal definitions shared by the HIP sources of libcola (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include "../../include/cola.h"

namespace cola {

constexpr int kThreads = 256;          // every kernel runs 4 waves of 64 lanes

typedef float  floatx4  __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8   __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// Per right-hand-side CG state (device memory, one per RHS of the current
// system).  Updated only by the last block of a reduction.
struct CgState {
    double rho;        // r.r of the current residual
    double alpha;      // rho / (p.Ap) of the current iteration
    double beta;       // rho_new / rho_old; 0 before the first direction
    double tol2;       // (tol * ||b||)^2 - stop when rho <= tol2
    double bnorm2;     // ||b||^2 of this solve's right-hand side
    double delta;      // reliable updates: replace r once ||r|| < delta * rmax (0: off)
    double rmax;       // ||r|| at the last reliable update
    double rho_true;   // ||b - A x||^2 from the latest FP64 residual
    int32_t active;    // 1 while iterating
    int32_t iters;
    int32_t status;    // COLA_* numerical status of this solve
    int32_t max_iters;
    int32_t need_update; // reliable update requested for the end of this chunk (kNoisePause: and
                         // paused until then, the recursion being at its noise floor)
    int32_t fails;     // consecutive reliable updates after which the true residual missed tol
    int32_t updates;   // reliable updates done
    int32_t restart_dir; // reliable updates restart the direction (p = r) instead of keeping it
    int32_t xdefer;    // x += alpha p is applied by the next iteration's first MVM pass, not the update
    int32_t xlag;      // (xdefer) x still lacks alpha p of the last step taken
    int32_t pbuf;      // which of two direction buffers holds the current p (pswap engines)
    int32_t pswap;     // the first MVM pass writes the new direction to the other buffer; the
                       // vector update then flips pbuf
};

// Reliable updates: a right-hand side whose recursive residual has fallen below kNoiseFloor
// times its last true residual stops iterating until the update at the end of its chunk
// (need_update = kNoisePause).  That far down, the FP32 recursion's residual and direction are
// made of rounding noise (orthogonality to the previous direction is lost), and further steps on
// them can make the residual grow without bound, e.g. for a right-hand side that is an
// eigenvector of the operator, whose residual is at the noise floor after one step.  A right-hand
// side falls this far within one chunk only when it converges that fast.
constexpr double kNoiseFloor = 1e-5;
constexpr int32_t kNoisePause = 2;

// Refinement (outer) state, one per RHS.
struct OuterState {
    double bnorm2;     // ||b||^2 of the caller's right-hand side (FP64)
    double rnorm;      // ||b - A x|| of the latest FP64 residual
    double prev_rnorm; // previous sweep's ||r|| (inf before the first)
    double relres;     // rnorm / ||b||
    double tol;        // target relative residual
    int32_t active;
    int32_t slow;      // consecutive sweeps that failed to halve ||r||
    int32_t sweeps;
    int32_t status;
    int32_t iters;     // inner iterations summed over sweeps
    int32_t max_sweeps;
};

// Residual history of a solve: row g (one right-hand side) of `data` receives the
// recursive relative residual after every `stride` iterations, `len` entries.
struct ResHist {
    double* data = nullptr;
    int32_t stride = 0;
    int32_t len = 0;
};

// Counters shared by all RHS of a solve (device memory).
struct SolveCounters {
    int32_t num_active;       // RHS still iterating in the current inner solve
    int32_t num_outer_active; // RHS still refining
};

// ---------------------------------------------------------------------------
// Wave / block reductions (fixed order, hence deterministic).
__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the 256 threads of a block; the result is valid in every thread.
__device__ inline double block_sum(double v, double* smem /* >= 4 doubles */) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) smem[wave] = v;
    __syncthreads();
    double s = smem[0] + smem[1] + smem[2] + smem[3];
    __syncthreads();
    return s;
}

// Coherent (L1-bypassing) accesses for data exchanged between blocks of one launch.
__device__ inline double load_coherent(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void store_coherent(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Last-block-done reduction: every block of a group publishes one partial;
// the block that arrives last sums the group's partials in index order and
// returns true (in all its threads) with the total in *total.  The counter
// is reset by that block so the next launch starts from zero.  No block ever
// waits for another, so the pattern cannot hang.
//
// Ordering without cache-wide fences: the partial is written with a relaxed
// device-scope atomic store (a coherent store that does not stay in this
// XCD's L2), the issuing thread waits for that store to complete, and only
// then increments the counter with a relaxed device-scope atomic.  The last
// block reads the partials with coherent atomic loads issued after it has
// seen the final count.  A release/acquire fence at device scope would
// instead write back and invalidate the whole L2 of the XCD from every
// block, which dominated the run time of the streaming kernels.
__device__ inline bool last_block_reduce(double partial, double* partials, uint32_t* counter,
                                         int nblocks, int myblock, double* total,
                                         double* smem) {
    __shared__ int s_last;
    if (threadIdx.x == 0) {
        store_coherent(&partials[myblock], partial);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);            // the partial store has completed
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const uint32_t prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == (uint32_t)(nblocks - 1));
    }
    __syncthreads();
    if (!s_last) return false;
    double s = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += blockDim.x) s += load_coherent(&partials[i]);
    s = block_sum(s, smem);
    if (threadIdx.x == 0)
        __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *total = s;
    return true;
}

// Block sum over the 8 waves of a GEMM block (fixed order); valid in every thread.
__device__ inline double block_sum8(double v, double* smem8) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) smem8[wave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < 8; ++w) t += smem8[w];
    __syncthreads();
    return t;
}

// The last-block-done reduction of common.h for 8-wave blocks.
__device__ inline bool last_block_reduce8(double partial, double* partials, uint32_t* counter, int nblocks,
                                          int myblock, double* total, double* smem8) {
    __shared__ int s_last;
    if (threadIdx.x == 0) {
        store_coherent(&partials[myblock], partial);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);            // the partial store has completed
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const uint32_t prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (prev == (uint32_t)(nblocks - 1));
    }
    __syncthreads();
    if (!s_last) return false;
    double t = 0.0;
    for (int i = threadIdx.x; i < nblocks; i += blockDim.x) t += load_coherent(&partials[i]);
    t = block_sum8(t, smem8);
    if (threadIdx.x == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    *total = t;
    return true;
}

// Residual history: every `stride` iterations the recursive relative residual sqrt(rho / ||b||^2)
// (the absolute one for b = 0) at entry iters / stride - 1 of this right-hand side's row.
__device__ inline void record_residual(const ResHist& h, int64_t g, const CgState& st, double rho) {
    if (!h.data || h.stride <= 0 || st.iters % h.stride != 0) return;
    const int k = st.iters / h.stride - 1;
    if (k < 0 || k >= h.len) return;
    h.data[g * h.len + k] = st.bnorm2 > 0.0 ? sqrt(rho / st.bnorm2) : sqrt(rho);
}

__device__ inline bool finite_d(double v) { return __builtin_isfinite(v); }

// Restarted refinement, after the FP64 residual of a sweep (||b - A x||^2 = tot): record it and
// decide the right-hand side's fate (converged, stagnated, out of sweeps, or refine again).
// Runs in one thread per right-hand side.
__device__ inline void outer_residual(OuterState& o, double tot, SolveCounters* cnt) {
    const double rn = sqrt(tot);
    const double bn = sqrt(o.bnorm2);
    o.rnorm = rn;
    o.relres = bn > 0.0 ? rn / bn : rn;
    int status = -100;   // still refining
    if (!finite_d(rn)) status = COLA_ERR_NONFINITE;
    else if (o.relres <= o.tol) status = COLA_OK;
    else {
        o.slow = (rn > 0.5 * o.prev_rnorm) ? o.slow + 1 : 0;
        if (o.slow >= 2) status = COLA_STAGNATED;
        else if (o.sweeps >= o.max_sweeps) status = COLA_NOT_CONVERGED;
    }
    o.prev_rnorm = rn;
    if (status != -100) {
        o.status = status;
        o.active = 0;
        atomicSub(&cnt->num_outer_active, 1);
    }
}

// After a reliable update has put ||b - A x||^2 into st.rho_true (x already
// holds the folded FP64 solution and r the replaced residual): decide
// convergence from the true residual, resume a paused right-hand side, and
// rescale beta so the next direction is r_new + (rho_true / rho_old) p (or
// restart it when the working precision is too coarse for the old one).
// Runs in one thread per right-hand side.
__device__ inline void reliable_finish(CgState& st, SolveCounters* cnt) {
    const double rt = st.rho_true;
    const bool was_active = st.active != 0;
    const bool noise_pause = st.need_update == kNoisePause;
    st.need_update = 0;
    st.updates += 1;
    bool run = false;
    if (!__builtin_isfinite(rt)) {
        st.status = COLA_ERR_NONFINITE;
    } else if (rt <= st.tol2) {
        st.status = COLA_OK;
    } else {
        // recursive residual converged, true one did not (a noise-floor pause is no convergence)
        if (!was_active && !noise_pause) st.fails += 1;
        else st.fails = 0;
        if (st.fails >= 3) st.status = COLA_STAGNATED;
        else if (st.iters >= st.max_iters) st.status = COLA_NOT_CONVERGED;
        else run = true;
        if (st.restart_dir) st.beta = 0.0;
        else if (st.rho > 0.0) st.beta = rt * st.beta / st.rho;
        st.rho = rt;
        st.rmax = sqrt(rt);
    }
    if (run && !was_active) {
        st.active = 1;
        atomicAdd(&cnt->num_active, 1);
    } else if (!run && was_active) {
        st.active = 0;
        atomicSub(&cnt->num_active, 1);
    }
}

// Row (within a 16x16 tile) of accumulator element v held by `lane`.  The
// column is always lane % 16.  FP32/BF16 16x16 MFMAs give each lane four
// consecutive rows; the FP64 16x16x4 MFMA interleaves them by 4.
__device__ inline int acc_row(float, int lane, int v)  { return 4 * (lane >> 4) + v; }
__device__ inline int acc_row(double, int lane, int v) { return 4 * v + (lane >> 4); }


// p_new = r + beta * p_old, evaluated identically wherever it is needed so
// that every kernel of an iteration sees the same rounded direction.
__device__ inline float  pnew_of(float r, float p, double beta)   { return __builtin_fmaf((float)beta, p, r); }
__device__ inline double pnew_of(double r, double p, double beta) { return __builtin_fma(beta, p, r); }

}  // namespace cola
