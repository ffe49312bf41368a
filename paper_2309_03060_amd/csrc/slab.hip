// Fused mode-2/mode-3 product of three-mode Kronecker terms.
//
// For a term K1 (x) K2 (x) K3 and X = x.reshape(n1, n2, n3), the mode-2 and
// mode-3 products act on each n2 x n3 slab X[i1] independently:
// T[i1] = K2 X[i1] K3^T (the per-mode evaluation behind the Kronecker MVM
// cost of Table 2).  When a slab fits in LDS (n2, n3 <= 64) both products
// are done there: the slab is read once, the intermediate product never
// leaves the CU, and T is written once.  Blocks are persistent over a range
// of slabs so the two factors are staged in LDS once per block, and the next
// slab's loads are issued while the current one is being multiplied.
#include "slab.h"

namespace cola {

// UP = 64 + 4 keeps the block at 52 KB of LDS (3 blocks per CU); a bank-free
// pitch of 80 for the second product's operand reads measured slower because
// it drops occupancy to 2 blocks.
struct SlabF32 { using V = float;  using Acc = floatx4;  static constexpr int KP = 64 + 4, UP = 64 + 4; };
struct SlabF64 { using V = double; using Acc = doublex4; static constexpr int KP = 64 + 2, UP = 64 + 2; };

__device__ inline floatx4 smma(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline doublex4 smma(double a, double b, doublex4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline void sload4(const float* p, float* o) {
    const floatx4 v = *(const floatx4*)p;
    o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
}
__device__ inline void sload4(const double* p, double* o) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 a = *(const d2*)p, b = *(const d2*)(p + 2);
    o[0] = a[0]; o[1] = a[1]; o[2] = b[0]; o[3] = b[1];
}
__device__ inline void sstore4(float* p, const float* v) { *(floatx4*)p = floatx4{v[0], v[1], v[2], v[3]}; }
__device__ inline void sstore4(double* p, const double* v) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    *(d2*)p = d2{v[0], v[1]};
    *(d2*)(p + 2) = d2{v[2], v[3]};
}

// FULL: 64 x 64 slabs (16-byte loads); PNEW: the slab is the CG direction
// r + beta p.  Both are template parameters so the prefetch below is
// straight-line code the compiler can leave in flight across the products.
template <class S, bool FULL, bool PNEW>
__global__ __launch_bounds__(kThreads) void k_slab23(SlabArgs a) {
    using V = typename S::V;
    using Acc = typename S::Acc;
    constexpr int D = 64, KP = S::KP, UP = S::UP;
    __shared__ __attribute__((aligned(16))) V K2s[D * KP];
    __shared__ __attribute__((aligned(16))) V K3s[D * KP];
    __shared__ __attribute__((aligned(16))) V Ut[D * UP];   // U = P K3^T (row-major), then the output T
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 15, lq = lane >> 4;
    const int n2 = a.n2, n3 = a.n3;
    const int64_t slab = (int64_t)n2 * n3;
    const int term = blockIdx.y;
    const V* K2 = (const V*)a.K2 + (int64_t)term * a.k2_tstride;
    const V* K3 = (const V*)a.K3 + (int64_t)term * a.k3_tstride;
    V* Yt = (V*)a.Y + (int64_t)term * a.y_tstride;
    const V* X = (const V*)a.X;
    const V* R = (const V*)a.R;
    constexpr bool full = FULL;

    for (int e = tid; e < D * D; e += kThreads) {
        const int r = e / D, c = e % D;
        K2s[r * KP + c] = (r < n2 && c < n2) ? K2[r * n2 + c] : (V)0;
        K3s[r * KP + c] = (r < n3 && c < n3) ? K3[r * n3 + c] : (V)0;
    }

    // The first product U = P K3^T is done per wave on a 16-row strip of the
    // slab, reading its A operand straight from global memory.  The inner
    // (column) index is permuted so each lane loads 4 consecutive columns at
    // once: at MFMA step s = 4u + c the lane group lq supplies column
    // 16u + 4 lq + c, and the B operand from K3 uses the same permutation.
    const int arow = 16 * wave + lr;             // slab row of this lane's A values
    V pv[16], rv[16];
    auto load_strip = [&](int64_t sl) {
        const int64_t base = sl * slab;
        if constexpr (FULL) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t off = base + arow * D + 16 * u + 4 * lq;
                sload4(X + off, pv + 4 * u);
                if constexpr (PNEW) sload4(R + off, rv + 4 * u);
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int col = 16 * u + 4 * lq + c;
                    const bool ok = arow < n2 && col < n3;
                    const int64_t off = base + (ok ? arow * n3 + col : 0);
                    pv[4 * u + c] = X[off];
                    if constexpr (PNEW) rv[4 * u + c] = R[off];
                    if (!ok) { pv[4 * u + c] = (V)0; if constexpr (PNEW) rv[4 * u + c] = (V)0; }
                }
        }
    };

    // Slabs are visited in grid-stride order.  The next slab's strip, gate
    // flag and direction coefficient are all loaded right after the first
    // product of the current slab, so they arrive while the second product
    // and the store run; a slab whose right-hand side is gated off is skipped
    // at the top of the loop (its loads were wasted, which only happens once
    // right-hand sides start to converge).
    auto beta_of = [&](int64_t s_) -> double { return PNEW ? a.cg[s_ / a.a_per_rhs].beta : 0.0; };
    // without a gate the flag is read from any valid address and ignored
    auto flag_of = [&](int64_t s_) -> int32_t {
        return *(a.gate ? a.gate + (s_ / a.a_per_rhs) * a.gate_stride : (const int32_t*)a.X);
    };
    auto next_active = [&](int64_t s_) -> int64_t {     // gate reads only
        while (s_ < a.nslabs && a.gate && !a.gate[(s_ / a.a_per_rhs) * a.gate_stride]) s_ += gridDim.x;
        return s_;
    };
    int64_t sl = blockIdx.x;
    int32_t flag = 0;
    double be = 0.0;
    __syncthreads();
    if (sl < a.nslabs) {
        load_strip(sl);
        flag = flag_of(sl);
        be = beta_of(sl);
    }
    while (sl < a.nslabs) {
        if (a.gate && !flag) {                     // gated off: find the next active slab first
            sl = next_active(sl + gridDim.x);
            if (sl < a.nslabs) {
                load_strip(sl);
                flag = 1;
                be = beta_of(sl);
            }
            continue;
        }
        const int64_t nx = sl + gridDim.x;
        const int64_t nxc = nx < a.nslabs ? nx : sl;          // clamped: the loads stay unconditional
        V av[16];
        if constexpr (PNEW) {
#pragma unroll
            for (int q = 0; q < 16; ++q) av[q] = pnew_of(rv[q], pv[q], be);
        } else {
#pragma unroll
            for (int q = 0; q < 16; ++q) av[q] = pv[q];
        }
        // U strip: rows 16 wave .. +15, all 64 columns (4 MFMA tiles)
        Acc acc1[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc1[j] = Acc{0, 0, 0, 0};
#pragma unroll
        for (int st = 0; st < 16; ++st) {
            const int kcol = 16 * (st >> 2) + 4 * lq + (st & 3);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc1[j] = smma(av[st], K3s[(16 * j + lr) * KP + kcol], acc1[j]);
        }
        load_strip(nxc);                           // next strip in flight during the second product
        const int32_t nx_flag = flag_of(nxc);
        const double nx_be = beta_of(nxc);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * wave + acc_row(acc1[j][v], lane, v);
                Ut[row * UP + 16 * j + lr] = (V)acc1[j][v];
            }
        __syncthreads();                           // U complete
        // T = K2 U  (T[b][c] = sum_a K2[b][a] U[a][c]); wave tile 32 x 32
        Acc acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = Acc{0, 0, 0, 0};
#pragma unroll 4
        for (int k = 0; k < D; k += 4) {
            V a2[2], b2[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a2[i] = K2s[(32 * wm + 16 * i + lr) * KP + k + lq];
#pragma unroll
            for (int j = 0; j < 2; ++j) b2[j] = Ut[(k + lq) * UP + 32 * wn + 16 * j + lr];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = smma(a2[i], b2[j], acc[i][j]);
        }
        __syncthreads();                           // U reads done
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 32 * wm + 16 * i + acc_row(acc[i][j][v], lane, v);
                    const int col = 32 * wn + 16 * j + lr;
                    Ut[row * UP + col] = (V)acc[i][j][v];
                }
        __syncthreads();
        const int64_t base = sl * slab;
        if (full) {
            for (int e = tid; e < D * D / 4; e += kThreads) {
                const int r = e / (D / 4), c = (e % (D / 4)) * 4;
                V v[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = Ut[r * UP + c + q];
                sstore4(Yt + base + r * D + c, v);
            }
        } else {
            for (int e = tid; e < slab; e += kThreads) Yt[base + e] = Ut[(e / n3) * UP + (e % n3)];
        }
        __syncthreads();                           // T read out of U before the next slab writes U
        sl = nx;
        flag = nx_flag;
        be = nx_be;
    }
}

bool slab_supported(int prec, int64_t n2, int64_t n3) {
    return (prec == COLA_PREC_FP32 || prec == COLA_PREC_FP64) && n2 >= 1 && n3 >= 1 && n2 <= 64 && n3 <= 64;
}

hipError_t launch_slab23(int prec, const SlabArgs& a, hipStream_t s) {
    const int64_t cap = (prec == COLA_PREC_FP64) ? 256 : 768;   // 1 (FP64) or 3 (FP32) blocks per CU
    const unsigned gx = (unsigned)(a.nslabs < cap ? a.nslabs : cap);
    dim3 grid(gx, (unsigned)a.nterms);
    const bool full = a.n2 == 64 && a.n3 == 64;
    const bool pn = a.pnew != 0;
#define COLA_SLAB_LAUNCH(S)                                                                              \
    do {                                                                                                 \
        if (full && pn) hipLaunchKernelGGL((k_slab23<S, true, true>), grid, dim3(kThreads), 0, s, a);    \
        else if (full) hipLaunchKernelGGL((k_slab23<S, true, false>), grid, dim3(kThreads), 0, s, a);    \
        else if (pn) hipLaunchKernelGGL((k_slab23<S, false, true>), grid, dim3(kThreads), 0, s, a);      \
        else hipLaunchKernelGGL((k_slab23<S, false, false>), grid, dim3(kThreads), 0, s, a);             \
    } while (0)
    if (prec == COLA_PREC_FP32) COLA_SLAB_LAUNCH(SlabF32);
    else if (prec == COLA_PREC_FP64) COLA_SLAB_LAUNCH(SlabF64);
    else return hipErrorInvalidValue;
#undef COLA_SLAB_LAUNCH
    return hipGetLastError();
}

}  // namespace cola
