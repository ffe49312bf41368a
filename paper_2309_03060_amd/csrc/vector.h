// Vector-phase kernels of CG and refinement: host launchers.
#pragma once
#include "common.h"

namespace cola {

int vec_blocks_per_rhs(int64_t n);

hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t fill_f64(double* p, double v, int64_t n, hipStream_t s);
hipError_t fill_f32(float* p, float v, int64_t n, hipStream_t s);
hipError_t copy_f64(const double* in, double* out, int64_t n, hipStream_t s);

// keep_x: X holds a warm start (left as it is) instead of being set to 0.
hipError_t outer_init(const double* B, double* X, int64_t n, int nrhs, OuterState* outer, double tol,
                      int max_sweeps, double* partials, int part_stride, uint32_t* counters,
                      SolveCounters* cnt, hipStream_t s, bool keep_x = false);

// keep_x: x holds a warm start and src = b - A x0; keep_bnorm: cg.bnorm2 already holds ||b||^2
// (rhs_norm2), so the tolerance stays relative to b.
template <typename T>
hipError_t cg_prepare(const double* src, T* r, T* x, T* p, int64_t n, int nrhs, const OuterState* outer,
                      CgState* cg, double tol, int max_iters, double delta, double* partials, int part_stride,
                      uint32_t* counters, SolveCounters* cnt, hipStream_t s, bool keep_x = false,
                      bool keep_bnorm = false);

// cg.bnorm2 = ||b||^2 per right-hand side.
hipError_t rhs_norm2(const double* B, int64_t n, int nrhs, CgState* cg, double* partials, int part_stride,
                     uint32_t* counters, hipStream_t s);

template <typename T>
hipError_t reliable_fold(double* x64, T* xlo, const T* p, const T* p2, int64_t n, int nrhs, const CgState* cg,
                         bool all_rhs, hipStream_t s);

template <typename T>
hipError_t reliable_apply(const double* r64, T* rlo, int64_t n, int nrhs, CgState* cg, double* partials,
                          int part_stride, uint32_t* counters, SolveCounters* cnt, hipStream_t s);

// hist (or null): per right-hand side g, hist_len (alpha, beta) pairs; iteration
// i (1-based) of g stores its step length and r.r ratio at pair i - 1.
// rh: the residual history (see ResHist), or an empty one.
template <typename T>
hipError_t cg_update(T* x, T* r, const T* p, const T* q, int64_t n, int nrhs, CgState* cg, double* partials,
                     int part_stride, uint32_t* counters, SolveCounters* cnt, hipStream_t s,
                     double* hist = nullptr, int hist_len = 0, ResHist rh = ResHist{});

template <typename T>
hipError_t refine_accumulate(double* x64, const T* d, int64_t n, int nrhs, const OuterState* outer,
                             hipStream_t s);

hipError_t outer_bookkeep(OuterState* outer, const CgState* cg, int nrhs, SolveCounters* cnt, hipStream_t s);
hipError_t write_info(cola_solve_info* info, const OuterState* outer, const CgState* cg, int nrhs, hipStream_t s);
hipError_t mark_unverified(CgState* cg, int nrhs, hipStream_t s);

hipError_t convert_f64_f32(const double* in, float* out, int64_t n, hipStream_t s);
hipError_t convert_f32_f64(const float* in, double* out, int64_t n, hipStream_t s);
hipError_t convert_f64_bf16_split(const double* in, __bf16* out, int64_t n, int nparts, int64_t plane,
                                  hipStream_t s);

}  // namespace cola
