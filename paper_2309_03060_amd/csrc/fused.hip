// Persistent fused CG for one-term three-mode FP32 operators with 64-wide modes.
//
// The separate-kernel path runs three launches per CG iteration (modes 2 and 3
// of the Kronecker MVM per slab, mode 1 with the direction update, the vector
// update) and moves q = A p through memory.  Here one cooperative launch runs
// many iterations.  Right-hand side g is owned by a group of `bpr` blocks that
// only ever exchange data with each other, so they meet at group barriers
// rather than grid-wide ones; each iteration has three phases:
//
//   A  per slab X[i1] (64 x 64): p = r + beta p (written back to p), then
//      T[i1] = K2 P[i1] K3^T  (modes 2 and 3, the per-mode evaluation behind
//      the Kronecker MVM cost of Table 2);
//   B  per column strip (64 rows i1 x 64 columns (i2, i3)): q = K1 T +
//      (sigma2 + d) p and the partial p.q; q stays in registers;
//   C  after the group sum of p.q gives alpha: r -= alpha q and the partial
//      r.r, whose group sum gives the convergence test and beta.
//
// The x update of an iteration is deferred to the next phase A, which reads
// the old p anyway (and to the end of the launch for the last iteration), so
// only q has to stay in registers.  Bytes per element and iteration: A reads
// r, p, x and writes p, T, x (24); B reads T, p (8); C reads and writes r (8):
// 40 against 56 for the separate kernels.  Data crossing blocks (p, T, r, the partial sums) is
// written and read with agent-coherent accesses (the cache-policy bit that
// the memory model uses for agent-scope atomics), so a barrier needs no cache
// write-back.  Each group barrier carries the block's part of the next group
// sum: a block posts its part once its shared stores are fenced, loads its own
// next operands (r for phase C, p for the next phase A), then polls the
// group's posts, which both waits and gathers.  The sums of a group are formed
// in one fixed order by every block of the group, so all of them take the
// same decisions without another barrier.
#include "fused.h"

#include <algorithm>

namespace cola {
namespace {

constexpr int D = 64;                      // mode size
constexpr int PD = D + 4;                  // LDS row pitch (floats)
constexpr int SL = D * D;                  // elements per slab and per strip
constexpr int NV = D * D * D;              // unknowns per right-hand side
constexpr int kFT = 1024;                  // threads per block: 4 quads of 4 waves
constexpr int kSC1 = 16;                   // cache-policy operand: agent-coherent access
constexpr uint32_t kSpinLimit = 1u << 22;  // barrier polls before a time-out (seconds)

typedef unsigned int uintx4 __attribute__((ext_vector_type(4)));

__device__ inline __amdgpu_buffer_rsrc_t vec_rsrc(const float* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, NV * 4, 0x00020000);
}
// Element offsets split into a per-lane part and a wave-uniform part (kept in
// a scalar register), so the addresses of an unrolled loop cost no registers.
__device__ inline floatx4 ldc(__amdgpu_buffer_rsrc_t rs, int lane_e, int uni_e) {
    return __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(rs, lane_e * 4, uni_e * 4, kSC1));
}
__device__ inline void stc(__amdgpu_buffer_rsrc_t rs, int lane_e, int uni_e, floatx4 v) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uintx4, v), rs, lane_e * 4, uni_e * 4, kSC1);
}
// The same through the ordinary cache path, for data only this block touches
// (x) or nobody writes (the diagonal); a resource of zero records reads zeros.
__device__ inline floatx4 ldn(__amdgpu_buffer_rsrc_t rs, int lane_e, int uni_e) {
    return __builtin_bit_cast(floatx4, __builtin_amdgcn_raw_buffer_load_b128(rs, lane_e * 4, uni_e * 4, 0));
}
__device__ inline void stn(__amdgpu_buffer_rsrc_t rs, int lane_e, int uni_e, floatx4 v) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uintx4, v), rs, lane_e * 4, uni_e * 4, 0);
}
__device__ inline floatx4 mma(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Sum over the 1024 threads of the block (valid in every thread).
__device__ inline double block_sum16(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kFT / 64; ++i) s += red[i];
    return s;
}

// This wave's memory operations have completed (stores included): issued by
// every wave that stored data other blocks read after the next barrier.
// The signal fences keep the compiler from moving memory operations across the wait.
__device__ inline void fence_stores() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Group barrier that carries one value per block.  Each group owns three
// sets of bpr slots, cycled by the barrier count k.  A slot holds a sentinel
// until its block posts a value; a block has arrived once its slot in set
// k mod 3 is not the sentinel, so polling the slots both waits and gathers
// the values (no counter, no second round trip).  After barrier k a block
// resets its own slot in set (k + 2) mod 3: every block read that set before
// arriving at barrier k, and the reset is fenced before the block's next post,
// so no block can see it stale at barrier k + 2.
constexpr uint64_t kSlotEmpty = ~0ull;                 // a NaN pattern arithmetic never makes

// Post this block's value (the caller's waves have fenced every store the
// group reads after the barrier).
__device__ inline void group_post(double v, double* gslots, int bpr, int rank, uint32_t k) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const double c = (v == v) ? v : __builtin_bit_cast(double, 0x7ff8000000000000ull);   // one NaN
        store_coherent(gslots + (k % 3) * bpr + rank, c);
    }
}

// Wait for the group and sum the posted values in a fixed butterfly order
// (the same total in every block).  Loads issued since the post stay in
// flight.  Returns false in every thread after a time-out (the flag is set;
// the launch is then void).
__device__ inline bool group_gather(double* gslots, int bpr, int rank, uint32_t k, uint32_t* err, double* s_tot,
                                    int* s_ok) {
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const double* set = gslots + (k % 3) * bpr;
        double v = 0.0;
        int ok = 1;
        for (uint32_t spins = 0;; ++spins) {
            v = lane < bpr ? load_coherent(set + lane) : 0.0;
            const bool ready = lane >= bpr || __builtin_bit_cast(uint64_t, v) != kSlotEmpty;
            if (__all(ready)) break;
            if (spins > kSpinLimit) {
                if (lane == 0) __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        v = wave_sum(v);
        if (lane == 0) {
            *s_tot = v;
            *s_ok = ok;
            store_coherent(gslots + ((k + 2) % 3) * bpr + rank, __builtin_bit_cast(double, kSlotEmpty));
        }
    }
    __syncthreads();
    return *s_ok != 0;
}

// CG scalars of the group's right-hand side, kept in LDS and updated by
// thread 0 (every block of the group computes the same values).
struct FState {
    double rho, beta, alpha;
    int iters, status, need_update, active;
    int pending;                  // x += alpha p of the last finished iteration not applied yet
};

// SPQ: slabs (phase A) and strips (phases B, C) per quad; a block owns 4 SPQ of each.
template <int SPQ>
__global__ __launch_bounds__(kFT) void k_fused_cg(FusedCgArgs a) {
    __shared__ __attribute__((aligned(16))) float K1s[D * PD];
    __shared__ __attribute__((aligned(16))) float K2s[D * PD];
    __shared__ __attribute__((aligned(16))) float K3s[D * PD];
    __shared__ __attribute__((aligned(16))) float Wq[4][D * PD];   // per-quad staging tile
    __shared__ double red[kFT / 64];
    __shared__ double s_tot;
    __shared__ int s_ok;
    __shared__ FState fs;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int quad = wave >> 2, qw = wave & 3, qt = tid & 255;
    const int lr = lane & 15, lq = lane >> 4, wm = qw >> 1, wn = qw & 1;
    // group g = blockIdx % nrhs: with round-robin dispatch the blocks of a group share an XCD
    const int grp = blockIdx.x % a.nrhs, rank = blockIdx.x / a.nrhs;
    CgState* stp = a.cg + grp;
    if (!stp->active) return;                       // the same decision in every block of the group
    const double tol2 = stp->tol2, delta = stp->delta, rmax = stp->rmax;
    const int max_iters = stp->max_iters;
    if (tid == 0) {
        fs.rho = stp->rho;
        fs.beta = stp->beta;
        fs.alpha = stp->alpha;
        fs.iters = stp->iters;
        fs.status = stp->status;
        fs.need_update = stp->need_update;
        fs.active = 1;
        fs.pending = 0;
    }

    const auto rsX = vec_rsrc(a.x + (int64_t)grp * NV);
    const auto rsD = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(a.dvec), (short)0,
                                                       a.dvec ? NV * 4 : 0, 0x00020000);
    const auto rsR = vec_rsrc(a.r + (int64_t)grp * NV);
    const auto rsP = vec_rsrc(a.p + (int64_t)grp * NV);
    const auto rsT = vec_rsrc(a.T + (int64_t)grp * NV);
    const float s2 = (float)a.sigma2;
    double* gslots = a.slots + (int64_t)grp * 3 * a.bpr;
    uint32_t k = 0;                                  // barriers passed in this launch

    for (int e = tid; e < D * D; e += kFT) {
        const int rr = e / D, c = e % D;
        K1s[rr * PD + c] = a.K1[e];
        K2s[rr * PD + c] = a.K2[e];
        K3s[rr * PD + c] = a.K3[e];
    }

    const int u0 = (rank * 4 + quad) * SPQ;          // this quad's first slab / strip
    float* Wt = Wq[quad];
    // phase A lane roles: row 16 qw + lr of the slab; the first product's k index
    // at step s = 4 u + c is column 16 u + 4 lq + c (4 consecutive columns per lane)
    const int arow = 16 * qw + lr;
    const int alane = arow * D + 4 * lq;            // + 16 u: this lane's elements of a slab
    // T write-out: float4 number qt + 256 q of a slab is row qt / 16 + 16 q, column 4 (qt % 16)
    const int tlane = (qt >> 4) * D + 4 * (qt & 15);
    const int tlds = (qt >> 4) * PD + 4 * (qt & 15);
    // phase B staging of a T strip: row qt / 4, columns 16 u + 4 (qt % 4) + c
    const int brow = qt >> 2, bsub = qt & 3;
    const int blane = brow * (D * D) + 4 * bsub;    // + 16 u (+ strip column c0)
    // phases B, C output roles: the transposed product Q^T = T^T K1^T puts 4 consecutive
    // columns of one output row in each lane; tile (ti, tj) of wave (wm, wn) holds row
    // 32 wn + 16 tj + lr, columns c0 + 32 wm + 16 ti + 4 lq + v
    const int olane = (32 * wn + lr) * (D * D) + 32 * wm + 4 * lq;   // + 16 ti (+ c0 + 16 D^2 tj)

    float pv[16], rv[16];                            // phase A operands of the current slab
    auto load_p = [&](int sl) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const floatx4 pp = ldc(rsP, alane + 16 * u, sl * SL);
#pragma unroll
            for (int c = 0; c < 4; ++c) pv[4 * u + c] = pp[c];
        }
    };
    auto load_r = [&](int sl) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const floatx4 r4 = ldc(rsR, alane + 16 * u, sl * SL);
#pragma unroll
            for (int c = 0; c < 4; ++c) rv[4 * u + c] = r4[c];
        }
    };
    load_p(u0);
    __syncthreads();                                 // factors staged, state initialised

    for (int it = 0; it < a.iters; ++it) {
        // ---------------- phase A ----------------
        // p = r + beta p per slab, with the previous iteration's x += alpha p
        // (deferred to here, where the old p is read anyway), then T = K2 P K3^T
        {
            const double beta = fs.beta;
            const float aprev = (float)fs.alpha;
            const bool pend = fs.pending != 0;
            load_r(u0);                              // p of the first slab is in flight already
#pragma unroll
            for (int s = 0; s < SPQ; ++s) {
                const int sl = u0 + s;
                floatx4 xv[4];                         // x arrives during the first product
#pragma unroll
                for (int u = 0; u < 4; ++u) xv[u] = ldn(rsX, alane + 16 * u, sl * SL);
                float av[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) av[q] = pnew_of(rv[q], pv[q], beta);
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    stc(rsP, alane + 16 * u, sl * SL, floatx4{av[4 * u], av[4 * u + 1], av[4 * u + 2], av[4 * u + 3]});
                floatx4 acc1[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) acc1[j] = floatx4{0, 0, 0, 0};
#pragma unroll
                for (int st = 0; st < 16; ++st) {
                    const int kcol = 16 * (st >> 2) + 4 * lq + (st & 3);
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc1[j] = mma(av[st], K3s[(16 * j + lr) * PD + kcol], acc1[j]);
                }
                if (pend) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
#pragma unroll
                        for (int c = 0; c < 4; ++c) xv[u][c] = __builtin_fmaf(aprev, pv[4 * u + c], xv[u][c]);
                        stn(rsX, alane + 16 * u, sl * SL, xv[u]);
                    }
                }
                if (s + 1 < SPQ) {                     // next slab in flight during the second product
                    load_p(sl + 1);
                    load_r(sl + 1);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v) Wt[(16 * qw + 4 * lq + v) * PD + 16 * j + lr] = acc1[j][v];
                __syncthreads();                               // U = P K3^T complete
                floatx4 acc[2][2];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0, 0, 0, 0};
#pragma unroll 4
                for (int k = 0; k < D; k += 4) {
                    float a2[2], b2[2];
#pragma unroll
                    for (int i = 0; i < 2; ++i) a2[i] = K2s[(32 * wm + 16 * i + lr) * PD + k + lq];
#pragma unroll
                    for (int j = 0; j < 2; ++j) b2[j] = Wt[(k + lq) * PD + 32 * wn + 16 * j + lr];
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int j = 0; j < 2; ++j) acc[i][j] = mma(a2[i], b2[j], acc[i][j]);
                }
                __syncthreads();                               // U reads done
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            Wt[(32 * wm + 16 * i + 4 * lq + v) * PD + 32 * wn + 16 * j + lr] = acc[i][j][v];
                __syncthreads();
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const floatx4 t4 = *(const floatx4*)(Wt + tlds + 16 * PD * q);
                    stc(rsT, tlane, sl * SL + 16 * D * q, t4);
                }
                __syncthreads();                               // T read out before the next slab
            }
        }
        if (tid == 0) fs.pending = 0;
        fence_stores();                                        // p and T visible to the group
        group_post(0.0, gslots, a.bpr, rank, k);
        if (!group_gather(gslots, a.bpr, rank, k++, a.err, &s_tot, &s_ok)) return;

        // ---------------- phase B ----------------
        // q = K1 T + (sigma2 + d) p per strip, computed transposed so each lane holds
        // 16-byte runs of q; q stays in registers for phase C
        floatx4 qh[SPQ][2][2];
        floatx4 rh[SPQ][2][2];
        double dot = 0.0;
        {
            floatx4 tv[4], pb[2][2];
            auto load_strip = [&](int s, floatx4* tv_, floatx4 (*pb_)[2]) {
                const int c0 = (u0 + s) * D;
#pragma unroll
                for (int u = 0; u < 4; ++u) tv_[u] = ldc(rsT, blane + 16 * u, c0);
#pragma unroll
                for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                    for (int tj = 0; tj < 2; ++tj) pb_[ti][tj] = ldc(rsP, olane + 16 * ti, c0 + 16 * SL * tj);
            };
            load_strip(0, tv, pb);
#pragma unroll
            for (int s = 0; s < SPQ; ++s) {
                const int c0 = (u0 + s) * D;
#pragma unroll
                for (int u = 0; u < 4; ++u) *(floatx4*)(Wt + brow * PD + 16 * u + 4 * bsub) = tv[u];
                __syncthreads();                               // T strip staged
                floatx4 tn[4], pn[2][2];
                if (s + 1 < SPQ) load_strip(s + 1, tn, pn);    // next strip in flight during this one
                floatx4 acc[2][2];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0, 0, 0, 0};
#pragma unroll 4
                for (int k = 0; k < D; k += 4) {
                    float ta[2], kb[2];
#pragma unroll
                    for (int ti = 0; ti < 2; ++ti) ta[ti] = Wt[(k + lq) * PD + 32 * wm + 16 * ti + lr];
#pragma unroll
                    for (int tj = 0; tj < 2; ++tj) kb[tj] = K1s[(32 * wn + 16 * tj + lr) * PD + k + lq];
#pragma unroll
                    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                        for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = mma(ta[ti], kb[tj], acc[ti][tj]);
                }
#pragma unroll
                for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                    for (int tj = 0; tj < 2; ++tj) {
                        const floatx4 d4 = ldn(rsD, olane + 16 * ti, c0 + 16 * SL * tj);
                        floatx4 q;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const float pe = pb[ti][tj][v];
                            q[v] = acc[ti][tj][v] + (s2 + d4[v]) * pe;
                            dot += (double)pe * (double)q[v];
                        }
                        qh[s][ti][tj] = q;
                    }
                if (s + 1 < SPQ) {
                    __syncthreads();                           // strip reads done before the next staging
#pragma unroll
                    for (int u = 0; u < 4; ++u) tv[u] = tn[u];
#pragma unroll
                    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                        for (int tj = 0; tj < 2; ++tj) pb[ti][tj] = pn[ti][tj];
                }
            }
        }
        const double dot_blk = block_sum16(dot, red);
        if (tid < 64) fence_stores();                          // the last slot reset (phase B stored nothing)
        group_post(dot_blk, gslots, a.bpr, rank, k);
        // r for phase C, in flight across the barrier
#pragma unroll
        for (int s = 0; s < SPQ; ++s)
#pragma unroll
            for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                for (int tj = 0; tj < 2; ++tj)
                    rh[s][ti][tj] = ldc(rsR, olane + 16 * ti, (u0 + s) * D + 16 * SL * tj);
        if (!group_gather(gslots, a.bpr, rank, k++, a.err, &s_tot, &s_ok)) return;
        if (tid == 0) {
            const double pq = s_tot;
            if (!(pq > 0.0) || !finite_d(pq)) {
                fs.status = finite_d(pq) ? COLA_ERR_NOT_SPD : COLA_ERR_NONFINITE;
                fs.active = 0;
                if (rank == 0) atomicSub(&a.cnt->num_active, 1);
            } else {
                fs.alpha = fs.rho / pq;
            }
        }
        __syncthreads();
        if (!fs.active) break;

        // ---------------- phase C ----------------
        // r -= alpha q and the partial r.r (x follows in the next phase A)
        const float af = (float)fs.alpha;
        double rr2 = 0.0;
#pragma unroll
        for (int s = 0; s < SPQ; ++s)
#pragma unroll
            for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                for (int tj = 0; tj < 2; ++tj) {
                    floatx4 r4 = rh[s][ti][tj];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        r4[v] = __builtin_fmaf(-af, qh[s][ti][tj][v], r4[v]);
                        rr2 += (double)r4[v] * (double)r4[v];
                    }
                    stc(rsR, olane + 16 * ti, (u0 + s) * D + 16 * SL * tj, r4);
                }
        const double rr_blk = block_sum16(rr2, red);
        fence_stores();                                        // r visible to the group
        group_post(rr_blk, gslots, a.bpr, rank, k);
        load_p(u0);                                            // the next phase A's own data, early
        if (!group_gather(gslots, a.bpr, rank, k++, a.err, &s_tot, &s_ok)) return;
        if (tid == 0) {
            // convergence, iteration limit and reliable-update request
            const double tot = s_tot;
            fs.iters += 1;
            fs.pending = 1;
            bool stop = true;
            if (!finite_d(tot)) {
                fs.status = COLA_ERR_NONFINITE;
            } else if (tot <= tol2) {
                if (delta > 0.0) fs.need_update = 1;
                else fs.status = COLA_OK;
            } else if (fs.iters >= max_iters) {
                fs.status = COLA_NOT_CONVERGED;
            } else {
                stop = false;
                if (delta > 0.0 && tot < delta * delta * rmax * rmax) {
                    fs.need_update = 1;
                    if (tot < kNoiseFloor * kNoiseFloor * rmax * rmax) {
                        fs.need_update = kNoisePause;
                        stop = true;
                    }
                }
            }
            fs.beta = tot / fs.rho;
            fs.rho = tot;
            if (stop) {
                fs.active = 0;
                if (rank == 0) atomicSub(&a.cnt->num_active, 1);
            }
        }
        __syncthreads();
        if (!fs.active) break;
    }
    // the last finished iteration's x += alpha p (its direction is still in p)
    if (fs.pending) {
        const float af = (float)fs.alpha;
#pragma unroll
        for (int s = 0; s < SPQ; ++s)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int sb = (u0 + s) * SL;
                const floatx4 p4 = ldc(rsP, alane + 16 * u, sb);
                floatx4 x4 = ldn(rsX, alane + 16 * u, sb);
#pragma unroll
                for (int c = 0; c < 4; ++c) x4[c] = __builtin_fmaf(af, p4[c], x4[c]);
                stn(rsX, alane + 16 * u, sb, x4);
            }
    }
    if (rank == 0 && tid == 0) {
        stp->rho = fs.rho;
        stp->alpha = fs.alpha;
        stp->beta = fs.beta;
        stp->iters = fs.iters;
        stp->status = fs.status;
        stp->need_update = fs.need_update;
        stp->active = fs.active;
    }
}

}  // namespace

bool fused_cg_supported(int prec, int Fv, int J, const int64_t* dims) {
    return prec == COLA_PREC_FP32 && Fv == 3 && J == 1 && dims[0] == D && dims[1] == D && dims[2] == D;
}

int fused_cg_max_blocks() {
    int dev = 0, coop = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    int p2 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_fused_cg<2>, kFT, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&p2, k_fused_cg<1>, kFT, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return std::min(per_cu, p2) * cus;
}

int fused_cg_blocks_per_rhs(int nrhs, int max_blocks) {
    if (max_blocks < 8) return 0;
    return (nrhs * 16 <= max_blocks) ? 16 : 8;
}

namespace {
__global__ void k_fused_report_timeout(const uint32_t* err, CgState* cg, int nrhs) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nrhs || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) return;
    cg[g].status = COLA_ERR_HIP;
    cg[g].active = 0;
    cg[g].need_update = 0;
}
}  // namespace

hipError_t fused_cg_report_timeout(const uint32_t* err, CgState* cg, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_fused_report_timeout, dim3((nrhs + 255) / 256), dim3(256), 0, s, err, cg, nrhs);
    return hipGetLastError();
}

hipError_t launch_fused_cg(const FusedCgArgs& a, hipStream_t s) {
    if (a.nrhs < 1 || (a.bpr != 8 && a.bpr != 16)) return hipErrorInvalidValue;
    FusedCgArgs args = a;
    void* kargs[] = {&args};
    const void* fn = a.bpr == 8 ? (const void*)k_fused_cg<2> : (const void*)k_fused_cg<1>;
    return hipLaunchCooperativeKernel(fn, dim3((unsigned)(a.nrhs * a.bpr)), dim3(kFT), kargs, 0, s);
}

}  // namespace cola
