// Fused mode-2/mode-3 product of three-mode Kronecker terms.
//
// For a term K1 (x) K2 (x) K3 and X = x.reshape(n1, n2, n3), the mode-2 and
// mode-3 products act on each n2 x n3 slab X[i1] independently:
// T[i1] = K2 X[i1] K3^T (the per-mode evaluation behind the Kronecker MVM
// cost of Table 2).  When a slab fits in LDS (n2, n3 <= 64) both products
// are done there: the slab is read once, the intermediate K2-free product
// never leaves the CU, and T is written once.  Blocks are persistent over a
// range of slabs so the two factors are staged in LDS once per block.
#include "slab.h"

namespace cola {

struct SlabF32 { using V = float;  using Acc = floatx4;  static constexpr int KP = 64 + 4; };
struct SlabF64 { using V = double; using Acc = doublex4; static constexpr int KP = 64 + 2; };

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

template <class S>
__global__ __launch_bounds__(kThreads) void k_slab23(SlabArgs a) {
    using V = typename S::V;
    using Acc = typename S::Acc;
    constexpr int D = 64, KP = S::KP;
    __shared__ __attribute__((aligned(16))) V K2s[D * KP];
    __shared__ __attribute__((aligned(16))) V K3s[D * KP];
    __shared__ __attribute__((aligned(16))) V Ps[D * KP];   // slab, later the output T
    __shared__ __attribute__((aligned(16))) V Ut[D * KP];   // (X K3^T) stored transposed
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int n2 = a.n2, n3 = a.n3;
    const int64_t slab = (int64_t)n2 * n3;
    const int term = blockIdx.y;
    const V* K2 = (const V*)a.K2 + (int64_t)term * a.k2_tstride;
    const V* K3 = (const V*)a.K3 + (int64_t)term * a.k3_tstride;
    V* Yt = (V*)a.Y + (int64_t)term * a.y_tstride;
    const V* X = (const V*)a.X;
    const V* R = (const V*)a.R;
    const bool full = (n2 == D && n3 == D);

    for (int e = tid; e < D * D; e += kThreads) {
        const int r = e / D, c = e % D;
        K2s[r * KP + c] = (r < n2 && c < n2) ? K2[r * n2 + c] : (V)0;
        K3s[r * KP + c] = (r < n3 && c < n3) ? K3[r * n3 + c] : (V)0;
    }

    for (int64_t sl = blockIdx.x; sl < a.nslabs; sl += gridDim.x) {
        const int64_t rhs = sl / a.a_per_rhs;
        if (a.gate && !a.gate[rhs * a.gate_stride]) continue;
        const double be = a.pnew ? a.cg[rhs].beta : 0.0;
        const int64_t base = sl * slab;
        __syncthreads();                     // previous slab's LDS reads are done
        if (full) {
            for (int e = tid; e < D * D / 4; e += kThreads) {
                const int r = e / (D / 4), c = (e % (D / 4)) * 4;
                V v[4];
                sload4(X + base + r * D + c, v);
                if (a.pnew) {
                    V rr[4];
                    sload4(R + base + r * D + c, rr);
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[q] = pnew_of(rr[q], v[q], be);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) Ps[r * KP + c + q] = v[q];
            }
        } else {
            for (int e = tid; e < D * D; e += kThreads) {
                const int r = e / D, c = e % D;
                V v = 0;
                if (r < n2 && c < n3) {
                    v = X[base + r * n3 + c];
                    if (a.pnew) v = pnew_of(R[base + r * n3 + c], v, be);
                }
                Ps[r * KP + c] = v;
            }
        }
        __syncthreads();
        // U = P K3^T  (U[a][c] = sum_k P[a][k] K3[c][k]); wave tile 32 x 32
        Acc acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = Acc{0, 0, 0, 0};
#pragma unroll 4
        for (int k = 0; k < D; k += 4) {
            V av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = Ps[(32 * wm + 16 * i + (lane & 15)) * KP + k + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < 2; ++j) bv[j] = K3s[(32 * wn + 16 * j + (lane & 15)) * KP + k + (lane >> 4)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = smma(av[i], bv[j], acc[i][j]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 32 * wm + 16 * i + acc_row(acc[i][j][v], lane, v);
                    const int col = 32 * wn + 16 * j + (lane & 15);
                    Ut[col * KP + row] = (V)acc[i][j][v];
                }
        __syncthreads();
        // T = K2 U  (T[b][c] = sum_a K2[b][a] U[a][c])
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = Acc{0, 0, 0, 0};
#pragma unroll 4
        for (int k = 0; k < D; k += 4) {
            V av[2], bv[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = K2s[(32 * wm + 16 * i + (lane & 15)) * KP + k + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < 2; ++j) bv[j] = Ut[(32 * wn + 16 * j + (lane & 15)) * KP + k + (lane >> 4)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = smma(av[i], bv[j], acc[i][j]);
        }
        // stage T row-major in Ps (P is no longer read), then write it out
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 32 * wm + 16 * i + acc_row(acc[i][j][v], lane, v);
                    const int col = 32 * wn + 16 * j + (lane & 15);
                    Ps[row * KP + col] = (V)acc[i][j][v];
                }
        __syncthreads();
        if (full) {
            for (int e = tid; e < D * D / 4; e += kThreads) {
                const int r = e / (D / 4), c = (e % (D / 4)) * 4;
                V v[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = Ps[r * KP + c + q];
                sstore4(Yt + base + r * D + c, v);
            }
        } else {
            for (int e = tid; e < n2 * n3; e += kThreads) {
                const int r = e / n3, c = e % n3;
                Yt[base + e] = Ps[r * KP + c];
            }
        }
    }
}

bool slab_supported(int prec, int64_t n2, int64_t n3) {
    return (prec == COLA_PREC_FP32 || prec == COLA_PREC_FP64) && n2 >= 1 && n3 >= 1 && n2 <= 64 && n3 <= 64;
}

hipError_t launch_slab23(int prec, const SlabArgs& a, hipStream_t s) {
    const int64_t cap = (prec == COLA_PREC_FP64) ? 256 : 512;
    const unsigned gx = (unsigned)(a.nslabs < cap ? a.nslabs : cap);
    dim3 grid(gx, (unsigned)a.nterms);
    if (prec == COLA_PREC_FP32)
        hipLaunchKernelGGL(k_slab23<SlabF32>, grid, dim3(kThreads), 0, s, a);
    else if (prec == COLA_PREC_FP64)
        hipLaunchKernelGGL(k_slab23<SlabF64>, grid, dim3(kThreads), 0, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace cola
