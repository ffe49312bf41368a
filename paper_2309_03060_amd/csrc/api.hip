// extern "C" entry points of libcola and the host-side drivers behind them.
//
// Everything numeric runs in the kernels of contract.hip / vector.hip /
// grad.hip; this file validates arguments, owns device memory, plans the
// per-mode passes of each Kronecker MVM and enqueues the CG and refinement
// loops on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include <rocprofiler-sdk-roctx/roctx.h>
#include <new>

#include "gemm.h"
#include "trace.h"
#include "eig.h"
#include "fused.h"
#include "gemm3.h"
#include "grad.h"
#include "op.h"
#include "resident.h"
#include "slab.h"
#include "small.h"
#include "pcg.h"
#include "slq.h"
#include "vector.h"

using namespace cola;

namespace cola {

int32_t dev_alloc(cola_op_s* op, void** p, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return COLA_ERR_OOM;
    }
    op->dev_sizes[*p] = bytes;
    op->dev_live += bytes;
    op->dev_peak = std::max(op->dev_peak, op->dev_live);
    return COLA_OK;
}

void dev_free(cola_op_s* op, void* p) {
    if (!p) return;
    auto it = op->dev_sizes.find(p);
    if (it != op->dev_sizes.end()) {
        op->dev_live -= it->second;
        op->dev_sizes.erase(it);
    }
    (void)hipFree(p);
}

}  // namespace cola

namespace {

#define HIP_TRY(expr)                                      \
    do {                                                   \
        hipError_t _e = (expr);                            \
        if (_e != hipSuccess) return COLA_ERR_HIP;         \
    } while (0)

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

void free_ws(cola_op_s* op) {
    Workspace& w = op->ws;
    void* ptrs[] = {w.vx, w.vr, w.vp, w.vq, w.inter[0], w.inter[1], w.r64, w.x64, w.b64, w.partials,
                    w.counters, w.cg, w.outer, w.cnt};
    for (void* p : ptrs)
        if (p) dev_free(op, p);
    if (w.host_flag) (void)hipHostFree(w.host_flag);
    w = Workspace();
}

// Blocks per right-hand side of the widest reduction any kernel may use.
int64_t max_blocks_per_rhs(const cola_op_s* op) {
    int64_t m = 512;
    for (const SysInfo& s : op->sys) {
        const int64_t B = s.n / s.dims[0];
        const int64_t b = ((B + 31) / 32) * ((s.dims[0] + 31) / 32);
        m = std::max(m, b);
        m = std::max<int64_t>(m, vec_blocks_per_rhs(s.n));
    }
    return m;
}

void destroy_graphs(cola_op_s* op);

int32_t ensure_ws(cola_op_s* op, int nrhs, hipStream_t st) {
    Workspace& w = op->ws;
    if (w.nrhs >= nrhs) return COLA_OK;
    destroy_graphs(op);
    free_ws(op);
    const size_t vec = (size_t)nrhs * (size_t)op->nmax * sizeof(double);
    int32_t rc = COLA_OK;
    rc |= dev_alloc(op, &w.vx, vec);
    rc |= dev_alloc(op, &w.vr, vec);
    rc |= dev_alloc(op, &w.vp, vec);
    rc |= dev_alloc(op, &w.vq, vec);
    rc |= dev_alloc(op, &w.inter[0], vec * op->Jmax);
    rc |= dev_alloc(op, &w.inter[1], vec * op->Jmax);
    rc |= dev_alloc(op, (void**)&w.r64, vec);
    rc |= dev_alloc(op, (void**)&w.x64, vec);
    rc |= dev_alloc(op, (void**)&w.b64, vec);
    w.part_stride = max_blocks_per_rhs(op);
    rc |= dev_alloc(op, (void**)&w.partials, sizeof(double) * (size_t)nrhs * w.part_stride);
    rc |= dev_alloc(op, (void**)&w.counters, sizeof(uint32_t) * (size_t)nrhs);
    rc |= dev_alloc(op, (void**)&w.cg, sizeof(CgState) * (size_t)nrhs);
    rc |= dev_alloc(op, (void**)&w.outer, sizeof(OuterState) * (size_t)nrhs);
    rc |= dev_alloc(op, (void**)&w.cnt, sizeof(SolveCounters));
    if (rc != COLA_OK) {
        free_ws(op);
        return COLA_ERR_OOM;
    }
    if (hipHostMalloc((void**)&w.host_flag, sizeof(int32_t) * 4, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        free_ws(op);
        return COLA_ERR_OOM;
    }
    w.nrhs = nrhs;
    HIP_TRY(fill_i32((int32_t*)w.counters, 0, nrhs, st));
    HIP_TRY(fill_i32((int32_t*)w.cnt, 0, 2, st));
    HIP_TRY(fill_i32((int32_t*)w.cg, 0, (int64_t)nrhs * sizeof(CgState) / 4, st));
    HIP_TRY(fill_i32((int32_t*)w.outer, 0, (int64_t)nrhs * sizeof(OuterState) / 4, st));
    return COLA_OK;
}

// ---------------------------------------------------------------------------
// tile choice: table entry (autotuned) or a size-based default
TileCfg tile_for(const cola_op_s* op, int prec, bool rows, int64_t nk, int64_t B, int64_t g) {
    auto it = op->tiles.find(PassKey{prec, rows ? 1 : 0, nk, B, g});
    if (it != op->tiles.end()) return it->second;
    if (rows) {
        const int wn = nk >= 64 ? 2 : 1;
        const int wm = g >= 8192 ? 4 : 2;
        return TileCfg{wm, wn};
    }
    const int wm = nk >= 128 ? 4 : (nk >= 48 ? 2 : 1);
    const int wn = B >= 128 ? 4 : (B >= 48 ? 2 : 1);
    return TileCfg{wm, wn};
}

struct ProfScope {
    Profiler* p; const char* name; hipStream_t s;
    ProfScope(Profiler& p_, const char* n, hipStream_t s_) : p(&p_), name(n), s(s_) { if (p->enabled) p->begin(name, s); }
    ProfScope(Profiler* p_, const char* n, hipStream_t s_) : p(p_), name(n), s(s_) {
        if (p && p->enabled) p->begin(name, s);
    }
    ~ProfScope() { if (p && p->enabled) p->end(name, s); }
};

const void* fac_base(const cola_op_s* op, int prec) {
    switch (prec) {
        case COLA_PREC_FP64: return op->fac64;
        case COLA_PREC_FP32: return op->fac32;
        default: return op->facbf;
    }
}

// Enqueue the passes of one MVM of system `s` on nrhs packed vectors `X`.
// The last pass (mode 1) applies epilogue `epi`; PassArgs fields for the
// epilogue and gating are taken from `tmpl`.  `inter` (two buffers of
// Jmax * nrhs * nmax working-precision elements each) holds the pass
// intermediates: the op's workspace, or the static scratch of the
// no-allocation product; `prof` (or null) times the launches.
int32_t enqueue_mvm(cola_op_s* op, const SysInfo& s, int prec, int nrhs, const void* X, const void* Rpnew,
                    void* Yout, const PassArgs& tmpl, hipStream_t st, void* const* inter, Profiler* prof) {
    const size_t esz = (prec == COLA_PREC_FP64) ? sizeof(double) : sizeof(float);
    const int64_t n = s.n;
    const int64_t tstride = (int64_t)nrhs * n;         // between per-term intermediates
    const void* fac = fac_base(op, prec);
    const int64_t k_plane = op->fac_elems;
    const void* diag = nullptr;
    if (s.diag_off >= 0)
        diag = (prec == COLA_PREC_FP64) ? (const void*)(op->diag64 + s.diag_off)
                                        : (const void*)(op->diag32 + s.diag_off);
    if (prec == COLA_PREC_FP64 && op->use_gemm64 && tmpl.epi != EPI_STORE && !tmpl.Ex &&
        gemm64_supported(s.Fv, s.dims) &&
        (tmpl.epi == EPI_MATVEC || gemm64_blocks_per_rhs(s.dims[0], s.dims[1]) <= tmpl.part_stride)) {
        // large two-mode operator in FP64 (residuals, FP64 CG, products): two dense FP64 GEMMs
        Gemm64Args g;
        std::memset(&g, 0, sizeof(g));
        g.n1 = (int32_t)s.dims[0];
        g.n2 = (int32_t)s.dims[1];
        g.J = s.J;
        g.nrhs = nrhs;
        g.U = op->fac64 + s.fac_off[0];
        g.V = op->fac64 + s.fac_off[1];
        const bool cg = tmpl.epi == EPI_CG;
        g.Pold = cg ? (const double*)X : nullptr;
        g.R = cg ? (const double*)Rpnew : nullptr;
        g.P = cg ? (double*)tmpl.Epout : nullptr;
        g.X = cg ? g.P : (const double*)X;
        g.Ep = cg ? g.P : (const double*)tmpl.Ep;
        g.Er = (const double*)tmpl.Er;
        g.T = (double*)inter[0];
        g.Y = (double*)Yout;
        g.dvec = (const double*)diag;
        g.sigma2 = s.sigma2;
        g.epi = tmpl.epi;
        g.cg = tmpl.cg;
        g.outer = tmpl.outer;
        g.gate = tmpl.gate;
        g.gate_stride = tmpl.gate_stride;
        g.partials = tmpl.partials;
        g.part_stride = tmpl.part_stride;
        g.counters = tmpl.counters;
        g.cnt = tmpl.cnt;
        auto al16 = [](const void* q) { return ((uintptr_t)q & 15) == 0; };
        if (al16(g.U) && al16(g.V) && al16(g.X) && al16(g.R) && al16(g.Pold) && al16(g.P) && al16(g.T) &&
            al16(g.Y) && al16(g.Ep) && al16(g.Er) && al16(g.dvec)) {
            if (cg) {
                ProfScope ps(prof, "gemm_pack_fp64", st);
                HIP_TRY(launch_gemm64(g, 0, st));
            }
            {
                ProfScope ps(prof, "gemm_mode2_fp64", st);
                HIP_TRY(launch_gemm64(g, 1, st));
            }
            {
                ProfScope ps(prof, "gemm_mode1_fp64", st);
                HIP_TRY(launch_gemm64(g, 2, st));
            }
            return COLA_OK;
        }
    }
    if (prec == COLA_PREC_FP64 && op->use_gemm64 && tmpl.epi != EPI_STORE && !tmpl.Ex &&
        gemm64_3_supported(s.Fv, s.J, s.dims) &&
        (tmpl.epi == EPI_MATVEC ||
         gemm64_3_blocks_per_rhs(s.dims[0], s.dims[1], s.dims[2]) <= tmpl.part_stride)) {
        // one-term three-mode operator in FP64: three dense FP64 GEMM passes, the last with the epilogue
        const int64_t n1 = s.dims[0], n2 = s.dims[1], n3 = s.dims[2];
        Gemm64Args g;
        std::memset(&g, 0, sizeof(g));
        g.J = 1;
        g.nrhs = nrhs;
        const bool cg = tmpl.epi == EPI_CG;
        g.Pold = cg ? (const double*)X : nullptr;
        g.R = cg ? (const double*)Rpnew : nullptr;
        g.P = cg ? (double*)tmpl.Epout : nullptr;
        g.Ep = cg ? g.P : (const double*)tmpl.Ep;
        g.Er = (const double*)tmpl.Er;
        g.dvec = (const double*)diag;
        g.sigma2 = s.sigma2;
        g.epi = tmpl.epi;
        g.cg = tmpl.cg;
        g.outer = tmpl.outer;
        g.gate = tmpl.gate;
        g.gate_stride = tmpl.gate_stride;
        g.partials = tmpl.partials;
        g.part_stride = tmpl.part_stride;
        g.counters = tmpl.counters;
        g.cnt = tmpl.cnt;
        const double* in3 = cg ? g.P : (const double*)X;
        auto al16 = [](const void* q) { return ((uintptr_t)q & 15) == 0; };
        const double* f3 = op->fac64 + s.fac_off[2];
        const double* f2 = op->fac64 + s.fac_off[1];
        const double* f1 = op->fac64 + s.fac_off[0];
        if (al16(in3) && al16(g.R) && al16(g.Pold) && al16(g.Ep) && al16(g.Er) && al16(g.dvec) && al16(Yout) &&
            al16(inter[0]) && al16(inter[1]) && al16(f1) && al16(f2) && al16(f3)) {
            if (cg) {
                Gemm64Args gp = g;
                gp.n1 = (int32_t)(n1 * n2);
                gp.n2 = (int32_t)n3;
                ProfScope ps(prof, "gemm_pack_fp64", st);
                HIP_TRY(launch_gemm64(gp, 0, st));
            }
            const char* names[3] = {"gemm_mode3_fp64", "gemm_mode2_fp64", "gemm_mode1_fp64"};
            for (int m = 3; m >= 1; --m) {
                Gemm64Args gm = g;
                if (m == 3) {
                    gm.n1 = (int32_t)(n1 * n2); gm.n2 = (int32_t)n3; gm.V = f3; gm.X = in3; gm.T = (double*)inter[0];
                } else if (m == 2) {
                    gm.n1 = (int32_t)(n3 * n1); gm.n2 = (int32_t)n2; gm.V = f2; gm.X = (const double*)inter[0];
                    gm.T = (double*)inter[1];
                } else {
                    gm.n1 = (int32_t)(n2 * n3); gm.n2 = (int32_t)n1; gm.V = f1; gm.X = (const double*)inter[1];
                    gm.Y = (double*)Yout;
                }
                ProfScope ps(prof, names[3 - m], st);
                HIP_TRY(launch_gemm64_pass(gm, m == 1, st));
            }
            return COLA_OK;
        }
    }
    if (op->use_gemm2 && (tmpl.epi == EPI_CG || tmpl.epi == EPI_MATVEC) && gemm2_supported(prec, s.Fv, s.dims)) {
        // large two-mode operator in BF16: both mode products as dense GEMMs
        Gemm2Args g;
        std::memset(&g, 0, sizeof(g));
        g.n1 = (int32_t)s.dims[0];
        g.n2 = (int32_t)s.dims[1];
        g.J = s.J;
        g.nrhs = nrhs;
        g.U = op->facbf + s.fac_off[0];
        g.V = op->facbf + s.fac_off[1];
        g.X = (const float*)X;
        g.R = (const float*)Rpnew;
        g.P = tmpl.epi == EPI_CG ? (float*)tmpl.Epout : nullptr;
        g.P16 = (__bf16*)inter[1];
        g.T = (__bf16*)inter[0];
        g.Y = (float*)Yout;
        g.dvec = (const float*)diag;
        g.sigma2 = s.sigma2;
        g.epi = tmpl.epi;
        g.cg = tmpl.cg;
        g.gate = tmpl.gate;
        g.gate_stride = tmpl.gate_stride;
        g.partials = tmpl.partials;
        g.part_stride = tmpl.part_stride;
        g.counters = tmpl.counters;
        g.cnt = tmpl.cnt;
        auto al16 = [](const void* q) { return ((uintptr_t)q & 15) == 0; };
        if (al16(g.U) && al16(g.V) && al16(g.X) && al16(g.R) && al16(g.P) && al16(g.Y) && al16(g.dvec)) {
            {
                ProfScope ps(prof, "gemm_pack", st);
                HIP_TRY(launch_gemm2(g, 0, st));
            }
            {
                ProfScope ps(prof, "gemm_mode2", st);
                HIP_TRY(launch_gemm2(g, 1, st));
            }
            {
                ProfScope ps(prof, "gemm_mode1", st);
                HIP_TRY(launch_gemm2(g, 2, st));
            }
            return COLA_OK;
        }
    }
    if (op->use_gemm3 && (tmpl.epi == EPI_CG || tmpl.epi == EPI_MATVEC) &&
        gemm3_supported(prec, s.Fv, s.J, s.dims)) {
        // one-term three-mode FP32 operator with 256-wide modes: three dense GEMMs
        Gemm3Args g;
        std::memset(&g, 0, sizeof(g));
        g.n1 = (int32_t)s.dims[0];
        g.n2 = (int32_t)s.dims[1];
        g.n3 = (int32_t)s.dims[2];
        g.nrhs = nrhs;
        g.K1 = op->fac32 + s.fac_off[0];
        g.K2 = op->fac32 + s.fac_off[1];
        g.K3 = op->fac32 + s.fac_off[2];
        g.bf16x3 = prec == COLA_PREC_BF16X3 ? 1 : 0;
        g.X = (const float*)X;
        g.R = (const float*)Rpnew;
        // the FP32 engine's direction pass also takes the deferred step x += alpha p_old; the BF16x3
        // engine (all modes 256) writes the new direction to a second buffer and takes the step in
        // its middle and last passes, else leaves x to the vector update
        const bool xsplit = g.bf16x3 && tmpl.epi == EPI_CG && tmpl.Ex && tmpl.Ep2 && g.n1 == kGemm3Tile &&
                            g.n2 == kGemm3Tile && g.n3 == kGemm3Tile;
        g.Xit = (tmpl.epi == EPI_CG && (!g.bf16x3 || xsplit)) ? (float*)tmpl.Ex : nullptr;
        g.P2 = xsplit ? (float*)tmpl.Ep2 : nullptr;
        g.Z1 = (float*)inter[0];
        g.Z2 = (float*)inter[1];
        g.Y = (float*)Yout;
        g.dvec = (const float*)diag;
        g.sigma2 = s.sigma2;
        g.epi = tmpl.epi;
        g.cg = tmpl.cg;
        g.gate = tmpl.gate;
        g.gate_stride = tmpl.gate_stride;
        g.partials = tmpl.partials;
        g.part_stride = tmpl.part_stride;
        g.counters = tmpl.counters;
        g.cnt = tmpl.cnt;
        auto al16 = [](const void* q) { return ((uintptr_t)q & 15) == 0; };
        const bool in_place_p = tmpl.epi != EPI_CG || tmpl.Epout == X;   // the direction is written over p_old
        if (in_place_p && al16(g.K1) && al16(g.K2) && al16(g.K3) && al16(g.X) && al16(g.R) &&
            al16(g.Xit) && al16(g.P2) && al16(g.Y) && al16(g.dvec)) {
            const char* names[3] = {"gemm_mode3", "gemm_mode2", "gemm_mode1"};
            for (int m = 3; m >= 1; --m) {
                ProfScope ps(prof, names[3 - m], st);
                HIP_TRY(launch_gemm3(g, m, st));
            }
            return COLA_OK;
        }
    }
    const void* in = X;
    int64_t in_tstride = 0;
    int buf = 0;
    int kstart = s.Fv - 1;
    if (s.Fv == 3 && op->use_slab && slab_supported(prec, s.dims[1], s.dims[2])) {
        // modes 3 and 2 of every term in one pass over n2 x n3 slabs
        const size_t fb = (prec == COLA_PREC_FP64) ? 8 : 4;
        SlabArgs sa;
        std::memset(&sa, 0, sizeof(sa));
        sa.nslabs = (int64_t)nrhs * s.dims[0];
        sa.a_per_rhs = s.dims[0];
        sa.n2 = (int32_t)s.dims[1];
        sa.n3 = (int32_t)s.dims[2];
        sa.nterms = s.J;
        sa.pnew = Rpnew != nullptr;
        sa.X = X;
        sa.R = Rpnew;
        sa.Y = inter[0];
        sa.y_tstride = tstride;
        sa.K2 = (const char*)fac + (size_t)s.fac_off[1] * fb;
        sa.K3 = (const char*)fac + (size_t)s.fac_off[2] * fb;
        sa.k2_tstride = s.dims[1] * s.dims[1];
        sa.k3_tstride = s.dims[2] * s.dims[2];
        sa.gate = tmpl.gate;
        sa.gate_stride = tmpl.gate_stride;
        sa.cg = tmpl.cg;
        {
            ProfScope ps(prof, prec == COLA_PREC_FP64 ? "slab23_fp64" : "slab23", st);
            HIP_TRY(launch_slab23(prec, sa, st));
        }
        in = inter[0];
        in_tstride = tstride;
        buf = 1;
        kstart = 0;
    }
    for (int k = kstart; k >= 0; --k) {
        PassArgs a = tmpl;
        const int64_t nk = s.dims[k];
        int64_t lead = 1, trail = 1;
        for (int m = 0; m < k; ++m) lead *= s.dims[m];
        for (int m = k + 1; m < s.Fv; ++m) trail *= s.dims[m];
        a.nk = (int32_t)nk;
        a.K = (const char*)fac + (size_t)s.fac_off[k] * (prec == COLA_PREC_FP64 ? 8 : (prec == COLA_PREC_FP32 ? 4 : 2));
        a.k_tstride = nk * nk;
        a.k_plane = k_plane;
        a.X = in;
        a.x_tstride = in_tstride;
        a.pnew = (k == s.Fv - 1) && Rpnew != nullptr;   // only the first pass forms the direction
        a.R = Rpnew;
        const bool rows = (k == s.Fv - 1);
        if (rows) {
            a.G = (int64_t)nrhs * lead;
            a.B = 1;
            a.a_per_rhs = lead;
        } else {
            a.G = (int64_t)nrhs * lead;
            a.B = trail;
            a.a_per_rhs = lead;
        }
        const char* kname;
        if (k == 0) {
            a.nsum = s.J;
            a.nout = 1;
            a.Y = Yout;
            a.y_tstride = 0;
            a.dvec = diag;
            a.sigma2 = s.sigma2;
            kname = prec == COLA_PREC_FP64 ? "contract_last_fp64" : "contract_last";
        } else {
            a.nsum = 1;
            a.nout = s.J;
            a.Y = inter[buf];
            a.y_tstride = tstride;
            a.epi = EPI_STORE;
            kname = prec == COLA_PREC_FP64 ? (rows ? "contract_rows_fp64" : "contract_mid_fp64")
                                           : (rows ? "contract_rows" : "contract_mid");
        }
        TileCfg cfg = tile_for(op, prec, rows, nk, a.B, a.a_per_rhs);
        {
            ProfScope ps(prof, kname, st);
            HIP_TRY(launch_contract(prec, rows, a, cfg, st));
        }
        in = a.Y;
        in_tstride = tstride;
        buf ^= 1;
        (void)esz;
    }
    return COLA_OK;
}

int32_t enqueue_mvm(cola_op_s* op, const SysInfo& s, int prec, int nrhs, const void* X, const void* Rpnew,
                    void* Yout, const PassArgs& tmpl, hipStream_t st) {
    return enqueue_mvm(op, s, prec, nrhs, X, Rpnew, Yout, tmpl, st, op->ws.inter, &op->prof);
}

PassArgs base_args(cola_op_s* op) {
    PassArgs a;
    std::memset(&a, 0, sizeof(a));
    a.partials = op->ws.partials;
    a.part_stride = (int32_t)op->ws.part_stride;
    a.counters = op->ws.counters;
    a.cnt = op->ws.cnt;
    return a;
}

int32_t poll_flag(cola_op_s* op, const int32_t* dev, hipStream_t st, int32_t* out) {
    HIP_TRY(hipMemcpyAsync(op->ws.host_flag, dev, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *out = *(volatile int32_t*)op->ws.host_flag;
    return COLA_OK;
}

// One CG iteration on prepared state (x, r, p, q are the working vectors):
// the MVM passes (direction update fused into the first and last pass) and
// the vector update.  defer_x: the MVM engine may take over x += alpha p
// (applied one iteration late by its first pass; reliable-update solves only,
// whose fold catches up a step still pending).
template <typename T>
int32_t enqueue_iteration(cola_op_s* op, const SysInfo& s, int prec, int nrhs, T* x, T* r, T* p, T* q,
                          bool defer_x, hipStream_t st) {
    Workspace& w = op->ws;
    PassArgs a = base_args(op);
    a.cg = w.cg;
    a.gate = &w.cg->active;
    a.gate_stride = (int32_t)(sizeof(CgState) / sizeof(int32_t));
    a.epi = EPI_CG;
    a.Ep = p;
    a.Er = r;
    a.Epout = p;
    a.Ex = defer_x ? x : nullptr;
    // the direction workspace holds 8 bytes per element: room for a second FP32 direction
    a.Ep2 = (defer_x && sizeof(T) == 4) ? (void*)(p + (int64_t)nrhs * s.n) : nullptr;
    int32_t rc = enqueue_mvm(op, s, prec, nrhs, p, r, q, a, st);
    if (rc != COLA_OK) return rc;
    ProfScope ps(op->prof, sizeof(T) == 8 ? "update_fp64" : "update", st);
    HIP_TRY(cg_update<T>(x, r, p, q, s.n, nrhs, w.cg, w.partials, (int)w.part_stride, w.counters, w.cnt, st,
                         sizeof(T) == 8 ? w.hist : nullptr, w.hist_len, w.rh));
    return COLA_OK;
}

// Reliable-update step appended to every chunk of a mixed-precision solve:
// for the right-hand sides that asked for it, fold x_lo into the FP64 x,
// form the FP64 residual b - A x (FP64 factors), and replace r_lo by it.
struct ReliableTail {
    double* X;        // FP64 solution (caller's buffer)
    const double* B;  // FP64 right-hand sides
    float* xl;        // low-precision iterate
    float* rl;        // low-precision residual
    const float* pl;  // low-precision direction (a deferred x += alpha p is caught up from it)
    const float* pl2; // its second buffer (the engines that alternate two direction buffers)
};

// final == false: the reliable update of the right-hand sides that asked for
// one (fold, FP64 residual, replace r and resume or finish).  final == true:
// after the last chunk, fold and form the FP64 residual only for the
// right-hand sides whose last true residual is stale (status not OK: iteration
// limit, breakdown); a converged one was certified by its last update and its
// x has not changed since.
int32_t enqueue_tail(cola_op_s* op, const SysInfo& s, int nrhs, const ReliableTail& t, bool final,
                     hipStream_t st) {
    TraceRange trace_range(final ? "reliable_final" : "reliable_update");
    Workspace& w = op->ws;
    if (final) HIP_TRY(mark_unverified(w.cg, nrhs, st));
    HIP_TRY(reliable_fold<float>(t.X, t.xl, t.pl, t.pl2, s.n, nrhs, w.cg, false, st));
    PassArgs a = base_args(op);
    a.cg = w.cg;
    a.gate = &w.cg->need_update;
    a.gate_stride = (int32_t)(sizeof(CgState) / sizeof(int32_t));
    a.epi = EPI_RESID_CG;
    a.Ep = t.X;
    a.Er = t.B;
    int32_t rc = enqueue_mvm(op, s, COLA_PREC_FP64, nrhs, t.X, nullptr, w.r64, a, st);
    if (rc != COLA_OK) return rc;
    if (!final)
        HIP_TRY(reliable_apply<float>(w.r64, t.rl, s.n, nrhs, w.cg, w.partials, (int)w.part_stride, w.counters,
                                      w.cnt, st));
    return COLA_OK;
}

void destroy_graphs(cola_op_s* op) {
    for (auto& kv : op->graphs) {
        for (int b = 0; b < 2; ++b) {
            if (kv.second.g[b].exec) (void)hipGraphExecDestroy(kv.second.g[b].exec);
            for (auto& e : kv.second.g[b].ev) {
                (void)hipEventDestroy(e.a);
                (void)hipEventDestroy(e.b);
            }
            if (kv.second.done[b]) (void)hipEventDestroy(kv.second.done[b]);
        }
    }
    op->graphs.clear();
}

// Capture `chunk` iterations into an executable graph (on the op's private
// capture stream; nothing executes during capture).
template <typename T>
int32_t capture_chunk(cola_op_s* op, const SysInfo& s, int prec, int nrhs, T* x, T* r, T* p, T* q, int chunk,
                      const ReliableTail* tail, ChunkGraph* out) {
    if (!op->cap_stream && hipStreamCreateWithFlags(&op->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return COLA_ERR_HIP;
    if (hipStreamBeginCapture(op->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return COLA_ERR_HIP;
    if (op->prof.enabled) op->prof.capture_list = &out->ev;
    int32_t rc = COLA_OK;
    for (int i = 0; i < chunk && rc == COLA_OK; ++i)
        rc = enqueue_iteration<T>(op, s, prec, nrhs, x, r, p, q, tail != nullptr, op->cap_stream);
    if (rc == COLA_OK && tail) rc = enqueue_tail(op, s, nrhs, *tail, false, op->cap_stream);
    op->prof.capture_list = nullptr;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(op->cap_stream, &g);
    if (rc != COLA_OK || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return rc != COLA_OK ? rc : COLA_ERR_HIP;
    }
    const hipError_t ie = hipGraphInstantiate(&out->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
        out->exec = nullptr;
        (void)hipGetLastError();
        return COLA_ERR_HIP;
    }
    return COLA_OK;
}

// Fused-CG workspace: barrier slots (which carry the group sums) and the time-out flag
// (allocated on the first fused solve; sized for every co-resident block).
int32_t ensure_fused(cola_op_s* op) {
    if (op->fused_max_blocks < 0) op->fused_max_blocks = fused_cg_max_blocks();
    if (op->fused_max_blocks < 8) return COLA_ERR_UNSUPPORTED;
    if (op->fused_slots) return COLA_OK;
    // three barrier-slot sets per block, then the time-out flag
    const size_t bytes = sizeof(double) * 3 * (size_t)op->fused_max_blocks + sizeof(uint32_t);
    int32_t rc = dev_alloc(op, (void**)&op->fused_slots, bytes);
    for (int b = 0; b < 2 && rc == COLA_OK; ++b)
        if (hipEventCreateWithFlags(&op->fused_done[b], hipEventDisableTiming) != hipSuccess) rc = COLA_ERR_HIP;
    if (rc == COLA_OK && hipMemset(op->fused_slots, 0, bytes) != hipSuccess) rc = COLA_ERR_HIP;
    if (rc != COLA_OK) {               // leave the path off rather than half set up
        (void)hipGetLastError();
        if (op->fused_slots) dev_free(op, op->fused_slots);
        op->fused_slots = nullptr;
        op->fused_max_blocks = 0;
    }
    return rc;
}

bool fused_eligible(const cola_op_s* op, const SysInfo& s, int prec, int check_every) {
    // the persistent kernel runs its own vector update, which records no residual history
    return op->use_fused && check_every >= 0 && op->fused_max_blocks != 0 && prec == op->prec && !op->ws.rh.data &&
           fused_cg_supported(prec, s.Fv, s.J, s.dims);
}

// CG iterations of a one-term three-mode FP32 operator with 64-wide modes:
// every chunk of check_every iterations is one cooperative launch per batch of
// right-hand sides (then the reliable-update tail), with the host reading the
// count of active right-hand sides one chunk behind, as in the graph path.
// check_every == 0: every chunk (128 iterations between reliable updates) is
// enqueued up front with no host wait, so the caller may capture the solve;
// groups that are no longer active leave a launch at once, and a barrier
// time-out is reported per right-hand side instead of by a host check.
int32_t run_cg_fused(cola_op_s* op, const SysInfo& s, int nrhs, float* x, float* r, float* p, int max_iters,
                     int check_every, const ReliableTail* tail, hipStream_t st) {
    Workspace& w = op->ws;
    const bool host_checks = check_every > 0;
    const int chunk = host_checks ? std::min(check_every, max_iters) : (tail ? std::min(128, max_iters) : max_iters);
    const int nchunks = (max_iters + chunk - 1) / chunk;
    const int bpr = fused_cg_blocks_per_rhs(nrhs, op->fused_max_blocks);
    const int per_launch = op->fused_max_blocks / bpr;
    const int64_t n = s.n;
    FusedCgArgs a{};
    a.bpr = bpr;
    a.iters = chunk;
    a.K1 = op->fac32 + s.fac_off[0];
    a.K2 = op->fac32 + s.fac_off[1];
    a.K3 = op->fac32 + s.fac_off[2];
    a.dvec = s.diag_off >= 0 ? op->diag32 + s.diag_off : nullptr;
    a.sigma2 = s.sigma2;
    a.slots = op->fused_slots;
    a.err = (uint32_t*)(op->fused_slots + 3 * (size_t)op->fused_max_blocks);
    a.cnt = w.cnt;
    float* t = (float*)w.inter[0];
    int last = -1;
    for (int c = 0; c < nchunks; ++c) {
        for (int g0 = 0; g0 < nrhs; g0 += per_launch) {
            a.nrhs = std::min(per_launch, nrhs - g0);
            a.x = x + g0 * n;
            a.r = r + g0 * n;
            a.p = p + g0 * n;
            a.T = t + g0 * n;
            a.cg = w.cg + g0;
            HIP_TRY(fill_i32((int32_t*)op->fused_slots, -1, (int64_t)a.nrhs * bpr * 3 * 2, st));   // all bits set
            ProfScope ps(op->prof, "cg_fused", st);
            const hipError_t le = launch_fused_cg(a, st);
            if (le != hipSuccess) {
                (void)hipGetLastError();
                // refused before any iteration ran: the caller continues on the separate-kernel path
                if (c == 0 && g0 == 0) {
                    op->use_fused = false;
                    return COLA_ERR_UNSUPPORTED;
                }
                return COLA_ERR_HIP;
            }
        }
        if (tail) {
            int32_t rc = enqueue_tail(op, s, nrhs, *tail, false, st);
            if (rc != COLA_OK) return rc;
        }
        if (!host_checks) continue;
        const int b = c & 1;
        HIP_TRY(hipMemcpyAsync(&w.host_flag[b], &w.cnt->num_active, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipEventRecord(op->fused_done[b], st));
        last = c;
        if (c >= 1) {
            HIP_TRY(hipEventSynchronize(op->fused_done[(c - 1) & 1]));
            if (*(volatile int32_t*)&w.host_flag[(c - 1) & 1] <= 0) break;
        }
    }
    if (!host_checks) {
        HIP_TRY(fused_cg_report_timeout(a.err, w.cg, nrhs, st));
        return COLA_OK;
    }
    if (last >= 0) HIP_TRY(hipEventSynchronize(op->fused_done[last & 1]));
    uint32_t timed_out = 0;
    HIP_TRY(hipMemcpy(&timed_out, a.err, sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (timed_out) {
        op->use_fused = false;         // a group never met: report it and stop using the path
        return COLA_ERR_HIP;
    }
    return COLA_OK;
}

// CG iterations.  check_every == 0: enqueue max_iters iterations directly
// (no host wait; safe under the caller's stream capture).  Otherwise the
// iterations run as replays of two captured chunk graphs of check_every
// iterations each; after launching chunk c the host waits for chunk c-1 and
// reads its count of still-active right-hand sides, so the device always has
// one chunk queued.  Iterations past convergence or past max_iters exit at
// once on the device.
template <typename T>
int32_t run_cg(cola_op_s* op, const SysInfo& s, int prec, int nrhs, T* x, T* r, T* p, T* q, int max_iters,
               int check_every, const ReliableTail* tail, hipStream_t st) {
    Workspace& w = op->ws;
    if constexpr (sizeof(T) == 4) {
        if (fused_eligible(op, s, prec, check_every) && ensure_fused(op) == COLA_OK) {
            const int32_t rc = run_cg_fused(op, s, nrhs, x, r, p, max_iters, check_every, tail, st);
            if (rc != COLA_ERR_UNSUPPORTED) return rc;
        }
    }
    const int chunk = check_every > 0 ? std::min(check_every, max_iters) : (tail ? std::min(32, max_iters) : max_iters);
    const int nchunks = (max_iters + chunk - 1) / chunk;
    auto direct_chunk = [&]() -> int32_t {
        for (int it = 0; it < chunk; ++it) {
            int32_t rc = enqueue_iteration<T>(op, s, prec, nrhs, x, r, p, q, tail != nullptr, st);
            if (rc != COLA_OK) return rc;
        }
        if (tail) return enqueue_tail(op, s, nrhs, *tail, false, st);
        return COLA_OK;
    };
    if (check_every <= 0) {
        for (int c = 0; c < nchunks; ++c) {
            int32_t rc = direct_chunk();
            if (rc != COLA_OK) return rc;
        }
        return COLA_OK;
    }
    GraphSet* gs = nullptr;
    if (op->graphs_ok) {
        GraphKey key{&s, prec, nrhs, x, r, p, q, chunk, (op->prof.enabled ? 1 : 0) + (tail ? 2 : 0),
                     op->tiles_version, sizeof(T) == 8 ? w.hist : nullptr, w.rh.data, w.rh.stride, w.rh.len};
        auto it = op->graphs.find(key);
        if (it == op->graphs.end() && op->graphs.size() >= 32) destroy_graphs(op);   // keep the cache bounded
        if (it == op->graphs.end()) {
            GraphSet set;
            int32_t rc = COLA_OK;
            for (int b = 0; b < 2 && rc == COLA_OK; ++b) {
                rc = capture_chunk<T>(op, s, prec, nrhs, x, r, p, q, chunk, tail, &set.g[b]);
                if (rc == COLA_OK && hipEventCreateWithFlags(&set.done[b], hipEventDisableTiming) != hipSuccess)
                    rc = COLA_ERR_HIP;
            }
            if (rc == COLA_OK) {
                it = op->graphs.emplace(key, set).first;
            } else {
                for (int b = 0; b < 2; ++b) {
                    if (set.g[b].exec) (void)hipGraphExecDestroy(set.g[b].exec);
                    for (auto& e : set.g[b].ev) {
                        (void)hipEventDestroy(e.a);
                        (void)hipEventDestroy(e.b);
                    }
                    if (set.done[b]) (void)hipEventDestroy(set.done[b]);
                }
                op->graphs_ok = false;     // fall back to direct launches from now on
            }
        }
        if (it != op->graphs.end()) gs = &it->second;
    }
    if (!gs) {
        for (int c = 0; c < nchunks; ++c) {
            if (c > 0) {
                int32_t active = 0;
                int32_t rc = poll_flag(op, &w.cnt->num_active, st, &active);
                if (rc != COLA_OK) return rc;
                if (active <= 0) break;
            }
            int32_t rc = direct_chunk();
            if (rc != COLA_OK) return rc;
        }
        return COLA_OK;
    }
    int last = -1;
    for (int c = 0; c < nchunks; ++c) {
        const int b = c & 1;
        HIP_TRY(hipGraphLaunch(gs->g[b].exec, st));
        HIP_TRY(hipMemcpyAsync(&w.host_flag[b], &w.cnt->num_active, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipEventRecord(gs->done[b], st));
        last = c;
        if (c >= 1) {
            const int pb = (c - 1) & 1;
            HIP_TRY(hipEventSynchronize(gs->done[pb]));
            if (op->prof.enabled) op->prof.harvest(gs->g[pb].ev);
            if (*(volatile int32_t*)&w.host_flag[pb] <= 0) break;
        }
    }
    if (last >= 0) {
        HIP_TRY(hipEventSynchronize(gs->done[last & 1]));
        if (op->prof.enabled) op->prof.harvest(gs->g[last & 1].ev);
    }
    return COLA_OK;
}

int32_t ensure_eig(cola_op_s* op, hipStream_t st);

// Scratch of the Kronecker-eigen transforms (at least `need` doubles).
int32_t ensure_eig_tmp(cola_op_s* op, int64_t need, hipStream_t st) {
    if (op->eig_tmp_elems >= need) return COLA_OK;
    (void)hipStreamSynchronize(st);
    if (op->eig_tmp) dev_free(op, op->eig_tmp);
    op->eig_tmp = nullptr;
    op->eig_tmp_elems = 0;
    if (dev_alloc(op, (void**)&op->eig_tmp, sizeof(double) * need) != COLA_OK) return COLA_ERR_OOM;
    op->eig_tmp_elems = need;
    return COLA_OK;
}

// One system's operator as plain pointers into the FP64 master copy.
DiagArgs diag_args(const cola_op_s* op, const SysInfo& s) {
    DiagArgs a;
    std::memset(&a, 0, sizeof(a));
    a.J = s.J;
    a.F = s.Fv;
    for (int k = 0; k < 3; ++k) {
        a.dims[k] = s.dims[k];
        a.fac[k] = k < s.Fv ? op->fac64 + s.fac_off[k] : nullptr;
    }
    a.dvec = s.diag_off >= 0 ? op->diag64 + s.diag_off : nullptr;
    a.sigma2 = s.sigma2;
    a.n = s.n;
    return a;
}

// Set up a preconditioner once per op: the Jacobi inverse diagonal of every
// system, or the first term's Kronecker eigendecomposition and the shift c of
// M = (first term) + c I per system (c = Tr(A - first term) / n).
int32_t ensure_precond(cola_op_s* op, int kind, hipStream_t st) {
    if (kind == COLA_PRECOND_JACOBI) {
        if (op->pc_dinv) return COLA_OK;
        double* dinv = nullptr;
        int32_t rc = dev_alloc(op, (void**)&dinv, sizeof(double) * op->n_total);
        if (rc != COLA_OK) return rc;
        for (const SysInfo& s : op->sys)
            if (kron_diagonal(diag_args(op, s), dinv + s.vec_off, true, st) != hipSuccess) {
                (void)hipGetLastError();
                (void)hipStreamSynchronize(st);
                dev_free(op, dinv);                        // not kept half filled
                return COLA_ERR_HIP;
            }
        op->pc_dinv = dinv;                                // published once every system is enqueued
        return COLA_OK;
    }
    int32_t rc = ensure_eig(op, st);
    if (rc != COLA_OK) return rc;
    if (op->pc_shift.size() == op->sys.size()) return COLA_OK;
    double* dev = op->ws.partials;                 // nsys doubles of scratch (before any solve uses it)
    std::vector<double> host(op->sys.size());
    for (size_t i = 0; i < op->sys.size(); ++i) {
        HIP_TRY(trace_shift(diag_args(op, op->sys[i]), dev, st));
        HIP_TRY(hipMemcpyAsync(&host[i], dev, sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    op->pc_shift = host;
    return COLA_OK;
}

// z = (first term + c I)^{-1} r for one system: two FP64 Kronecker MVMs with the
// eigenvector factors and one scaling by 1 / (eigenvalue products + c).
int32_t apply_kron_eig(cola_op_s* op, size_t si, int nrhs, const double* r, double* z, hipStream_t st) {
    const SysInfo& s = op->sys[si];
    double* y = op->eig_tmp;
    for (int step = 0; step < 2; ++step) {
        cola_op_s* sub = step == 0 ? op->eig_qt : op->eig_q;
        int32_t rc = ensure_ws(sub, nrhs, st);
        if (rc != COLA_OK) return rc;
        PassArgs a = base_args(sub);
        a.epi = EPI_MATVEC;
        a.Ep = step == 0 ? (const void*)r : (const void*)y;
        rc = enqueue_mvm(sub, sub->sys[si], COLA_PREC_FP64, nrhs, a.Ep, nullptr, step == 0 ? (void*)y : (void*)z,
                         a, st);
        if (rc != COLA_OK) return rc;
        if (step == 0) {
            const double* lam[3] = {nullptr, nullptr, nullptr};
            for (int k = 0; k < s.Fv; ++k) lam[k] = op->eig_lam + op->eig_lam_off[si][k];
            HIP_TRY(eig_scale(y, y, nrhs, s.Fv, s.dims, lam, op->pc_shift[si], st));
        }
    }
    return COLA_OK;
}

// r64 = B - A x with the FP64 factors for every right-hand side, ||r64||^2 into cg.rho_true.
int32_t true_residual(cola_op_s* op, const SysInfo& s, const double* B, const double* x, int nrhs,
                      hipStream_t st) {
    Workspace& w = op->ws;
    PassArgs a = base_args(op);
    a.cg = w.cg;
    a.epi = EPI_RESID_CG;
    a.Ep = x;
    a.Er = B;
    return enqueue_mvm(op, s, COLA_PREC_FP64, nrhs, x, nullptr, w.r64, a, st);
}

// Warm start of an FP64 CG: x = x0 (the caller's X), r0 = B - A x0 in r64, ||B||^2 in cg.bnorm2;
// cg_prepare then starts from src = r64 keeping x and the norm.
int32_t warm_start64(cola_op_s* op, const SysInfo& s, const double* B, const double* X0, double* x, int nrhs,
                     hipStream_t st) {
    Workspace& w = op->ws;
    HIP_TRY(copy_f64(X0, x, (int64_t)nrhs * s.n, st));
    HIP_TRY(rhs_norm2(B, s.n, nrhs, w.cg, w.partials, (int)w.part_stride, w.counters, st));
    return true_residual(op, s, B, x, nrhs, st);
}

// Preconditioned CG in FP64 (textbook recurrence): the MVM pass forms
// p = z + beta p and the step length as in plain CG, the update kernel moves x
// and r and decides convergence on ||r||, then z = M^{-1} r and r.z give the
// next beta.  Direct launches; the host polls the active count every
// check_every iterations.
int32_t run_pcg(cola_op_s* op, const SysInfo& s, const double* B, double* X, int nrhs, const cola_solve_opts* o,
                cola_solve_info* info, hipStream_t st) {
    Workspace& w = op->ws;
    const int64_t n = s.n;
    const int ps = (int)w.part_stride;
    const size_t si = (size_t)(&s - op->sys.data());
    int32_t rc = ensure_precond(op, o->precond, st);
    if (rc != COLA_OK) return rc;
    if (o->precond == COLA_PRECOND_KRON_EIG) {
        rc = ensure_eig_tmp(op, (int64_t)nrhs * n, st);
        if (rc != COLA_OK) return rc;
    }
    double* x = (double*)w.vx;
    double* r = (double*)w.vr;
    double* p = (double*)w.vp;
    double* q = (double*)w.vq;
    double* z = w.r64;
    const double* dinv = o->precond == COLA_PRECOND_JACOBI ? op->pc_dinv + s.vec_off : nullptr;
    const int vb = vec_blocks_per_rhs(n);
    auto precondition = [&]() -> int32_t {
        if (!dinv) {
            const int32_t rc2 = apply_kron_eig(op, si, nrhs, r, z, st);
            if (rc2 != COLA_OK) return rc2;
        }
        ProfScope ps2(op->prof, "pcg_precond_dot", st);
        HIP_TRY(pcg_precond_dot(r, z, dinv, n, nrhs, w.cg, w.partials, ps, w.counters, w.cnt, vb, st));
        return COLA_OK;
    };
    HIP_TRY(fill_i32(&w.cnt->num_active, 0, 1, st));
    const bool warm = o->x0_given && X;
    if (warm) {
        rc = warm_start64(op, s, B, X, x, nrhs, st);      // r0 in r64, which z reuses after the prepare
        if (rc != COLA_OK) return rc;
    }
    HIP_TRY(cg_prepare<double>(warm ? w.r64 : B, r, x, p, n, nrhs, nullptr, w.cg, o->tol, o->max_iters, 0.0,
                               w.partials, ps, w.counters, w.cnt, st, warm, warm));
    rc = precondition();
    if (rc != COLA_OK) return rc;
    for (int it = 0; it < o->max_iters; ++it) {
        if (o->check_every > 0 && it > 0 && it % o->check_every == 0) {
            int32_t active = 0;
            rc = poll_flag(op, &w.cnt->num_active, st, &active);
            if (rc != COLA_OK) return rc;
            if (active <= 0) break;
        }
        PassArgs a = base_args(op);
        a.cg = w.cg;
        a.gate = &w.cg->active;
        a.gate_stride = (int32_t)(sizeof(CgState) / sizeof(int32_t));
        a.epi = EPI_CG;
        a.Ep = p;
        a.Er = z;
        a.Epout = p;
        rc = enqueue_mvm(op, s, COLA_PREC_FP64, nrhs, p, z, q, a, st);
        if (rc != COLA_OK) return rc;
        {
            ProfScope ps2(op->prof, "pcg_update", st);
            HIP_TRY(pcg_update(x, r, p, q, n, nrhs, w.cg, w.partials, ps, w.counters, w.cnt, vb, st, w.rh));
        }
        rc = precondition();
        if (rc != COLA_OK) return rc;
    }
    HIP_TRY(pcg_finish(w.cg, nrhs, st));
    rc = true_residual(op, s, B, x, nrhs, st);            // relres_true of the returned x
    if (rc != COLA_OK) return rc;
    if (X) HIP_TRY(copy_f64(x, X, (int64_t)nrhs * n, st));
    if (info) HIP_TRY(write_info(info, nullptr, w.cg, nrhs, st));
    return COLA_OK;
}

int32_t solve_system(cola_op_s* op, const SysInfo& s, const double* B, double* X, int nrhs,
                     const cola_solve_opts* o, cola_solve_info* info, hipStream_t st) {
    TraceRange trace_range("solve_system");
    Workspace& w = op->ws;
    const int64_t n = s.n;
    const int ps = (int)w.part_stride;
    if (o->prec == COLA_PREC_FP64 && o->precond != COLA_PRECOND_NONE)
        return run_pcg(op, s, B, X, nrhs, o, info, st);
    if (o->prec == COLA_PREC_FP64) {
        HIP_TRY(fill_i32(&w.cnt->num_active, 0, 1, st));
        double* r = (double*)w.vr;
        double* p = (double*)w.vp;
        double* q = (double*)w.vq;
        double* x = (double*)w.vx;     // workspace iterate: captured graphs never hold caller pointers
        const bool warm = o->x0_given && X;
        if (warm) {
            int32_t rc = warm_start64(op, s, B, X, x, nrhs, st);
            if (rc != COLA_OK) return rc;
        }
        HIP_TRY(cg_prepare<double>(warm ? w.r64 : B, r, x, p, n, nrhs, nullptr, w.cg, o->tol, o->max_iters, 0.0,
                                   w.partials, ps, w.counters, w.cnt, st, warm, warm));
        int32_t rc = run_cg<double>(op, s, COLA_PREC_FP64, nrhs, x, r, p, q, o->max_iters, o->check_every, nullptr,
                                    st);
        if (rc != COLA_OK) return rc;
        rc = true_residual(op, s, B, x, nrhs, st);       // relres_true of the returned x
        if (rc != COLA_OK) return rc;
        if (X) HIP_TRY(copy_f64(x, X, (int64_t)nrhs * n, st));
        if (info) HIP_TRY(write_info(info, nullptr, w.cg, nrhs, st));
        return COLA_OK;
    }
    float* xl = (float*)w.vx;
    float* rl = (float*)w.vr;
    float* pl = (float*)w.vp;
    float* ql = (float*)w.vq;
    if (o->refine == COLA_REFINE_RELIABLE) {
        // one low-precision CG whose residual is replaced by the FP64 true
        // residual whenever it has dropped by inner_tol (reliable updates)
        // the FP64 solution and right-hand side live in the workspace so the
        // captured chunk graphs never hold caller pointers
        const bool warm = o->x0_given && X;
        if (warm) HIP_TRY(copy_f64(X, w.x64, (int64_t)nrhs * n, st));
        else HIP_TRY(fill_f64(w.x64, 0.0, (int64_t)nrhs * n, st));
        HIP_TRY(copy_f64(B, w.b64, (int64_t)nrhs * n, st));
        HIP_TRY(fill_i32(&w.cnt->num_active, 0, 1, st));
        if (warm) {
            // the low-precision CG solves for the correction to x0: its right-hand side is
            // r0 = b - A x0 (FP64), its tolerance stays relative to ||b||
            HIP_TRY(rhs_norm2(w.b64, n, nrhs, w.cg, w.partials, ps, w.counters, st));
            int32_t rc = true_residual(op, s, w.b64, w.x64, nrhs, st);
            if (rc != COLA_OK) return rc;
        }
        // plain BF16 operands: restart the direction at each update (signalled by a negative delta)
        const double delta = (op->prec == COLA_PREC_BF16) ? -o->inner_tol : o->inner_tol;
        HIP_TRY(cg_prepare<float>(warm ? w.r64 : w.b64, rl, xl, pl, n, nrhs, nullptr, w.cg, o->tol, o->max_iters,
                                  delta, w.partials, ps, w.counters, w.cnt, st, false, warm));
        ReliableTail tail{w.x64, w.b64, xl, rl, pl, pl + (int64_t)nrhs * n};
        int32_t rc = run_cg<float>(op, s, op->prec, nrhs, xl, rl, pl, ql, o->max_iters, o->check_every, &tail, st);
        if (rc != COLA_OK) return rc;
        rc = enqueue_tail(op, s, nrhs, tail, true, st);       // final fold and true residual where stale
        if (rc != COLA_OK) return rc;
        HIP_TRY(copy_f64(w.x64, X, (int64_t)nrhs * n, st));
        if (info) HIP_TRY(write_info(info, nullptr, w.cg, nrhs, st));
        return COLA_OK;
    }
    // restarted iterative refinement: FP64 residual, working-precision inner CG
    HIP_TRY(fill_i32(&w.cnt->num_outer_active, 0, 1, st));
    HIP_TRY(outer_init(B, X, n, nrhs, w.outer, o->tol, o->max_sweeps, w.partials, ps, w.counters, w.cnt, st,
                       o->x0_given != 0));
    for (int sweep = 0; sweep <= o->max_sweeps; ++sweep) {
        PassArgs a = base_args(op);
        a.outer = w.outer;
        a.gate = &w.outer->active;
        a.gate_stride = (int32_t)(sizeof(OuterState) / sizeof(int32_t));
        a.epi = EPI_RESID;
        a.Ep = X;
        a.Er = B;
        int32_t rc = enqueue_mvm(op, s, COLA_PREC_FP64, nrhs, X, nullptr, w.r64, a, st);
        if (rc != COLA_OK) return rc;
        if (sweep == o->max_sweeps) break;
        if (o->check_every > 0) {
            int32_t active = 0;
            rc = poll_flag(op, &w.cnt->num_outer_active, st, &active);
            if (rc != COLA_OK) return rc;
            if (active <= 0) break;
        }
        HIP_TRY(fill_i32(&w.cnt->num_active, 0, 1, st));
        HIP_TRY(cg_prepare<float>(w.r64, rl, xl, pl, n, nrhs, w.outer, w.cg, o->inner_tol, o->max_iters, 0.0,
                                  w.partials, ps, w.counters, w.cnt, st));
        rc = run_cg<float>(op, s, op->prec, nrhs, xl, rl, pl, ql, o->max_iters, o->check_every, nullptr, st);
        if (rc != COLA_OK) return rc;
        HIP_TRY(refine_accumulate<float>(X, xl, n, nrhs, w.outer, st));
        HIP_TRY(outer_bookkeep(w.outer, w.cg, nrhs, w.cnt, st));
    }
    if (info) HIP_TRY(write_info(info, w.outer, nullptr, nrhs, st));
    return COLA_OK;
}

void free_resident(cola_op_s* op) {
    void* ptrs[] = {op->res_sys, op->res_order, op->res_x, op->res_r, op->res_p, op->res_t64, op->res_st,
                    op->res_queue};
    for (void* p : ptrs)
        if (p) dev_free(op, p);
    op->res_sys = nullptr;
    op->res_order = nullptr;
    op->res_x = op->res_r = op->res_p = nullptr;
    op->res_t64 = nullptr;
    op->res_st = nullptr;
    op->res_queue = nullptr;
    op->res_nrhs = 0;
}

int32_t ensure_resident(cola_op_s* op, int nrhs, hipStream_t st) {
    if (op->res_nrhs >= nrhs && op->res_nrhs == nrhs) return COLA_OK;
    free_resident(op);
    const int nsys = (int)op->sys.size();
    const int64_t nitems = (int64_t)nsys * nrhs;
    const size_t vec = (size_t)nrhs * op->n_total;
    int32_t rc = COLA_OK;
    rc |= dev_alloc(op, &op->res_sys, sizeof(ResSys) * nsys);
    rc |= dev_alloc(op, (void**)&op->res_order, sizeof(int32_t) * nitems);
    rc |= dev_alloc(op, (void**)&op->res_x, sizeof(float) * vec);
    rc |= dev_alloc(op, (void**)&op->res_r, sizeof(float) * vec);
    rc |= dev_alloc(op, (void**)&op->res_p, sizeof(float) * vec);
    rc |= dev_alloc(op, (void**)&op->res_t64, sizeof(double) * vec);
    rc |= dev_alloc(op, (void**)&op->res_st, sizeof(CgState) * nitems);
    rc |= dev_alloc(op, (void**)&op->res_queue, sizeof(uint32_t) * 4);
    if (rc != COLA_OK) {
        free_resident(op);
        return COLA_ERR_OOM;
    }
    std::vector<ResSys> hs(nsys);
    for (int i = 0; i < nsys; ++i) {
        const SysInfo& s = op->sys[i];
        ResSys& r = hs[i];
        r.n1 = (int32_t)s.dims[0];
        r.n2 = (int32_t)s.dims[1];
        r.n = s.n;
        r.vec_off = s.vec_off;
        r.k1_off = s.fac_off[0];
        r.k2_off = s.fac_off[1];
        r.diag_off = s.diag_off;
        r.sigma2 = s.sigma2;
    }
    // largest systems first: the longest solves start early (LPT order)
    std::vector<int32_t> order(nitems);
    for (int64_t i = 0; i < nitems; ++i) order[i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return op->sys[x / nrhs].n > op->sys[y / nrhs].n;
    });
    // synchronous uploads: this runs once per (op, nrhs), outside any capture
    if (hipMemcpy(op->res_sys, hs.data(), sizeof(ResSys) * nsys, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(op->res_order, order.data(), sizeof(int32_t) * nitems, hipMemcpyHostToDevice) != hipSuccess) {
        free_resident(op);
        return COLA_ERR_HIP;
    }
    HIP_TRY(fill_i32((int32_t*)op->res_st, 0, nitems * (int64_t)sizeof(CgState) / 4, st));
    op->res_nrhs = nrhs;
    return COLA_OK;
}

// All systems at once through the resident kernel: rounds of (persistent FP32
// CG until each item needs a reliable update) + (FP64 residual of the items
// that asked), then one FP64 residual of every item for the final report.
int32_t solve_resident(cola_op_s* op, const double* B, double* X, int nrhs, const cola_solve_opts* o,
                       cola_solve_info* info, hipStream_t st) {
    int32_t rc = ensure_ws(op, 1, st);              // counters and pinned poll flag
    if (rc != COLA_OK) return rc;
    rc = ensure_resident(op, nrhs, st);
    if (rc != COLA_OK) return rc;
    Workspace& w = op->ws;
    ResArgs a;
    std::memset(&a, 0, sizeof(a));
    a.sys = (const ResSys*)op->res_sys;
    a.order = op->res_order;
    a.nitems = (int32_t)(op->sys.size() * nrhs);
    a.nrhs = nrhs;
    a.queue = op->res_queue;
    a.fac32 = op->fac32;
    a.fac64 = op->fac64;
    a.diag32 = op->diag32;
    a.diag64 = op->diag64;
    a.x = op->res_x;
    a.r = op->res_r;
    a.p = op->res_p;
    a.x64 = X;
    a.b64 = B;
    a.t64 = op->res_t64;
    a.st = op->res_st;
    a.cnt = w.cnt;
    HIP_TRY(fill_i32(&w.cnt->num_active, 0, 1, st));
    HIP_TRY(launch_resident_prepare(a, o->tol, o->max_iters, o->inner_tol, st));
    const int grid = std::max(1, std::min(a.nitems, op->num_cus > 0 ? op->num_cus : 256));
    const int rounds = std::max(o->max_sweeps, 32);
    for (int rd = 0; rd < rounds; ++rd) {
        if (o->check_every > 0 && rd > 0) {
            int32_t active = 0;
            rc = poll_flag(op, &w.cnt->num_active, st, &active);
            if (rc != COLA_OK) return rc;
            if (active <= 0) break;
        }
        HIP_TRY(fill_i32((int32_t*)op->res_queue, 0, 1, st));
        {
            ProfScope ps(op->prof, "resident", st);
            HIP_TRY(launch_resident_cg(a, grid, st));
        }
        HIP_TRY(launch_resident_resid64(a, st));
    }
    a.all_items = 1;
    HIP_TRY(launch_resident_resid64(a, st));
    if (info) HIP_TRY(write_info(info, nullptr, op->res_st, a.nitems, st));
    return COLA_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// FP64 solves of small one-term two-mode systems: one workgroup per (system, RHS)
// runs the whole CG; the per-system descriptors are built on the first call.
// Per-system descriptors of the one-workgroup FP64 kernel (built when the op is created).
int32_t build_small(cola_op_s* op) {
    const int nsys = (int)op->sys.size();
    std::vector<ResSys> h(nsys);
    for (int i = 0; i < nsys; ++i) {
        const SysInfo& s = op->sys[i];
        h[i].n1 = (int32_t)s.dims[0];
        h[i].n2 = (int32_t)s.dims[1];
        h[i].n = s.n;
        h[i].vec_off = s.vec_off;
        h[i].k1_off = s.fac_off[0];
        h[i].k2_off = s.fac_off[1];
        h[i].diag_off = s.diag_off;
        h[i].sigma2 = s.sigma2;
    }
    int32_t rc = dev_alloc(op, &op->small_sys, sizeof(ResSys) * nsys);
    if (rc != COLA_OK) return rc;
    if (hipMemcpy(op->small_sys, h.data(), sizeof(ResSys) * nsys, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        return COLA_ERR_HIP;
    }
    return COLA_OK;
}

int32_t solve_small(cola_op_s* op, const double* B, double* X, int nrhs, const cola_solve_opts* o,
                    cola_solve_info* info, hipStream_t st) {
    const int nsys = (int)op->sys.size();
    SmallArgs a;
    std::memset(&a, 0, sizeof(a));
    a.sys = (const ResSys*)op->small_sys;
    a.nitems = nsys * nrhs;
    a.nrhs = nrhs;
    a.fac64 = op->fac64;
    a.diag64 = op->diag64;
    a.B = B;
    a.X = X;
    a.tol = o->tol;
    a.max_iters = o->max_iters;
    a.info = info;
    a.x0_given = o->x0_given ? 1 : 0;
    if (o->hist && o->hist_stride > 0 && o->hist_len > 0) {
        a.rh.data = o->hist;
        a.rh.stride = o->hist_stride;
        a.rh.len = o->hist_len;
    }
    ProfScope ps(op->prof, "small_cg64", st);
    HIP_TRY(launch_small_cg64(a, st));
    return COLA_OK;
}

// ---------------------------------------------------------------------------
// Static scratch of the no-allocation product (cola_kron_matvec_noalloc): the two
// pass intermediates live in this array instead of the op's workspace.  Each GPU
// the library runs on holds its own copy from module load to process end.  In
// host code `scratch` names a host-side stand-in, never device memory: its device
// address comes from hipGetSymbolAddress, once per device, and only that address
// is used (kernel arguments).
constexpr size_t kScratchBytes = (size_t)64 << 20;   // two halves of 32 MiB
constexpr int kMaxDevices = 64;
__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of this device's scratch (device `dev` must be current).
int32_t scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return COLA_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return COLA_ERR_HIP;
        }
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return COLA_OK;
}

int32_t check_opts(const cola_op_s* op, const cola_solve_opts* o) {
    if (!o) return COLA_ERR_INVALID_ARG;
    if (!finite_pos(o->tol) || o->max_iters < 1 || o->check_every < 0) return COLA_ERR_INVALID_ARG;
    if (o->precond < COLA_PRECOND_NONE || o->precond > COLA_PRECOND_KRON_EIG) return COLA_ERR_INVALID_ARG;
    if (o->precond != COLA_PRECOND_NONE && o->prec != COLA_PREC_FP64) return COLA_ERR_UNSUPPORTED;
    if (o->hist && (o->hist_stride < 1 || o->hist_len < 1)) return COLA_ERR_INVALID_ARG;
    if (o->prec != COLA_PREC_FP64) {
        if (o->prec != op->prec) return COLA_ERR_INVALID_ARG;
        if (!finite_pos(o->inner_tol) || o->inner_tol >= 1.0) return COLA_ERR_INVALID_ARG;
        if (o->refine != COLA_REFINE_RELIABLE && o->refine != COLA_REFINE_RESTART) return COLA_ERR_INVALID_ARG;
        if (o->refine == COLA_REFINE_RESTART && o->max_sweeps < 1) return COLA_ERR_INVALID_ARG;
    }
    return COLA_OK;
}

}  // namespace

// ===========================================================================
extern "C" {

const char* cola_status_string(int32_t status) {
    switch (status) {
        case COLA_OK: return "ok";
        case COLA_NOT_CONVERGED: return "not converged: iteration or sweep limit reached";
        case COLA_STAGNATED: return "stagnated: refinement stopped reducing the residual";
        case COLA_ERR_INVALID_ARG: return "invalid argument";
        case COLA_ERR_NOT_SPD: return "operator not positive definite (CG breakdown p^T A p <= 0)";
        case COLA_ERR_NONFINITE: return "non-finite value (NaN/Inf) in the data or the iteration";
        case COLA_ERR_OOM: return "device memory allocation failed";
        case COLA_ERR_HIP: return "HIP runtime error";
        case COLA_ERR_UNSUPPORTED: return "unsupported configuration";
        case COLA_ERR_SCRATCH:
            return "call too large for the static scratch of the no-allocation product (64 MiB: "
                   "terms x nrhs x largest system x element size must not exceed 32 MiB)";
        default: return "unknown status";
    }
}

int32_t cola_op_create(const cola_system_desc* systems, int32_t nsys, int32_t prec, void* stream,
                       cola_op_t* out) {
    TraceRange trace_range("cola_op_create");
    if (!out) return COLA_ERR_INVALID_ARG;
    *out = nullptr;
    if (!systems || nsys < 1) return COLA_ERR_INVALID_ARG;
    if (prec < COLA_PREC_FP64 || prec > COLA_PREC_BF16X3) return COLA_ERR_INVALID_ARG;
    cola_op_s* op = new (std::nothrow) cola_op_s();
    if (!op) return COLA_ERR_OOM;
    op->prec = prec;
    (void)hipGetDevice(&op->device);
    hipStream_t st = S(stream);

    int64_t fac = 0, dg = 0, voff = 0, goff = 0;
    for (int i = 0; i < nsys; ++i) {
        const cola_system_desc& d = systems[i];
        if (d.nterms < 1 || d.nfactors < 1 || d.nfactors > 3 || !d.factors || !std::isfinite(d.sigma2) ||
            d.sigma2 < 0.0) {
            delete op;
            return COLA_ERR_INVALID_ARG;
        }
        SysInfo s;
        s.J = d.nterms;
        s.F = d.nfactors;
        s.Fv = std::max(2, s.F);
        int64_t n = 1;
        for (int k = 0; k < s.F; ++k) {
            if (d.dims[k] < 1 || d.dims[k] > (1 << 20)) {
                delete op;
                return COLA_ERR_INVALID_ARG;
            }
            n *= d.dims[k];
        }
        if (n > ((int64_t)1 << 36)) {
            delete op;
            return COLA_ERR_INVALID_ARG;
        }
        if (s.F == 1) {
            s.dims[0] = 1;
            s.dims[1] = d.dims[0];
        } else {
            for (int k = 0; k < s.F; ++k) s.dims[k] = d.dims[k];
        }
        for (int j = 0; j < s.J * s.F; ++j)
            if (!d.factors[j]) {
                delete op;
                return COLA_ERR_INVALID_ARG;
            }
        s.n = n;
        for (int k = 0; k < s.Fv; ++k) {
            s.fac_off[k] = fac;
            fac += (int64_t)s.J * s.dims[k] * s.dims[k];
        }
        if (d.diag) {
            s.diag_off = dg;
            dg += n;
        }
        s.sigma2 = d.sigma2;
        s.vec_off = voff;
        voff += n;
        s.grad_off = goff;
        goff += (int64_t)s.J * s.F;
        op->sys.push_back(s);
        op->nmax = std::max(op->nmax, n);
        op->Jmax = std::max(op->Jmax, s.J);
    }
    op->n_total = voff;
    op->fac_elems = fac;
    op->diag_elems = dg;
    // many small two-mode single-term systems go through the resident batched kernel
    op->resident_ok = (prec == COLA_PREC_FP32) && nsys >= 2;
    for (const SysInfo& s : op->sys)
        if (s.F != 2 || s.J != 1 || s.dims[0] > kResMax || s.dims[1] > kResMax) op->resident_ok = false;
    // small one-term two-mode systems: whole FP64 solves in one workgroup each
    bool small_ok = true;
    for (const SysInfo& s : op->sys)
        if (s.Fv != 2 || s.J != 1 || s.dims[0] > kSmallMax || s.dims[1] > kSmallMax) small_ok = false;
    (void)hipDeviceGetAttribute(&op->num_cus, hipDeviceAttributeMultiprocessorCount, op->device);

    int32_t rc = dev_alloc(op, (void**)&op->fac64, sizeof(double) * fac);
    if (rc == COLA_OK && dg > 0) rc = dev_alloc(op, (void**)&op->diag64, sizeof(double) * dg);
    if (rc != COLA_OK) {
        cola_op_destroy(op);
        return rc;
    }
    // copy factors into the packed FP64 master (mode-major, then term)
    for (int i = 0; i < nsys; ++i) {
        const cola_system_desc& d = systems[i];
        const SysInfo& s = op->sys[i];
        for (int k = 0; k < s.Fv; ++k) {
            const int64_t nk = s.dims[k];
            for (int j = 0; j < s.J; ++j) {
                double* dst = op->fac64 + s.fac_off[k] + (int64_t)j * nk * nk;
                hipError_t e;
                if (s.F == 1 && k == 0) {
                    e = fill_f64(dst, 1.0, 1, st);               // the implicit [1] factor
                } else {
                    const int kk = (s.F == 1) ? 0 : k;
                    e = hipMemcpyAsync(dst, d.factors[j * s.F + kk], sizeof(double) * nk * nk,
                                       hipMemcpyDeviceToDevice, st);
                }
                if (e != hipSuccess) {
                    cola_op_destroy(op);
                    return COLA_ERR_HIP;
                }
            }
        }
        if (d.diag && hipMemcpyAsync(op->diag64 + s.diag_off, d.diag, sizeof(double) * s.n,
                                     hipMemcpyDeviceToDevice, st) != hipSuccess) {
            cola_op_destroy(op);
            return COLA_ERR_HIP;
        }
    }
    op->small_ok = small_ok && build_small(op) == COLA_OK;
    // working copies
    if (prec != COLA_PREC_FP64) {
        rc = dev_alloc(op, (void**)&op->fac32, sizeof(float) * fac);
        if (rc == COLA_OK && dg > 0) rc = dev_alloc(op, (void**)&op->diag32, sizeof(float) * dg);
        if (rc == COLA_OK && (prec == COLA_PREC_BF16 || prec == COLA_PREC_BF16X3)) {
            op->nsplit = (prec == COLA_PREC_BF16) ? 1 : 3;
            rc = dev_alloc(op, (void**)&op->facbf, sizeof(__bf16) * fac * op->nsplit);
        }
        if (rc != COLA_OK) {
            cola_op_destroy(op);
            return rc;
        }
        if (convert_f64_f32(op->fac64, op->fac32, fac, st) != hipSuccess ||
            (dg > 0 && convert_f64_f32(op->diag64, op->diag32, dg, st) != hipSuccess) ||
            (op->facbf && convert_f64_bf16_split(op->fac64, op->facbf, fac, op->nsplit, fac, st) != hipSuccess)) {
            cola_op_destroy(op);
            return COLA_ERR_HIP;
        }
    }
    *out = op;
    return COLA_OK;
}

// ---------------------------------------------------------------------------
// Kronecker-eigen solve: decompose every factor once (FP64 one-sided Jacobi),
// keep the eigenvector factors as two internal operators (Q^T and Q) and the
// eigenvalues; a solve is then two Kronecker MVMs and one scaling.
namespace {
int32_t ensure_eig(cola_op_s* op, hipStream_t st) {
    if (op->eig_q) return COLA_OK;
    int64_t nmax = 1, lam_total = 0, vec_total = 0;
    op->eig_lam_off.assign(op->sys.size(), {0, 0, 0});
    for (size_t i = 0; i < op->sys.size(); ++i) {
        const SysInfo& s = op->sys[i];
        for (int k = 0; k < s.Fv; ++k) {
            nmax = std::max(nmax, s.dims[k]);
            op->eig_lam_off[i][k] = lam_total;
            lam_total += s.dims[k];
            vec_total += s.dims[k] * s.dims[k];
        }
    }
    double *vt = nullptr, *q = nullptr, *work = nullptr, *off = nullptr;
    int32_t rc = dev_alloc(op, (void**)&op->eig_lam, sizeof(double) * lam_total);
    rc |= dev_alloc(op, (void**)&vt, sizeof(double) * vec_total);
    rc |= dev_alloc(op, (void**)&q, sizeof(double) * vec_total);
    rc |= dev_alloc(op, (void**)&work, sizeof(double) * nmax * nmax);
    rc |= dev_alloc(op, (void**)&off, sizeof(double) * 2);
    auto cleanup = [&]() {
        for (void* p : {(void*)vt, (void*)q, (void*)work, (void*)off})
            if (p) dev_free(op, p);
    };
    if (rc != COLA_OK) {
        (void)hipStreamSynchronize(st);
        cleanup();
        dev_free(op, op->eig_lam);                         // a later call starts from scratch
        op->eig_lam = nullptr;
        return COLA_ERR_OOM;
    }
    std::vector<std::array<const void*, 3>> fqt(op->sys.size()), fq(op->sys.size());
    std::vector<cola_system_desc> dqt(op->sys.size()), dq(op->sys.size());
    int64_t voff = 0;
    for (size_t i = 0; i < op->sys.size() && rc == COLA_OK; ++i) {
        const SysInfo& s = op->sys[i];
        for (int k = 0; k < s.Fv && rc == COLA_OK; ++k) {
            const int64_t nk = s.dims[k];
            rc = jacobi_eig(op->fac64 + s.fac_off[k], nk, vt + voff, op->eig_lam + op->eig_lam_off[i][k], work,
                            off, 4e-15, 40, st);
            if (rc == COLA_OK && transpose_f64(vt + voff, q + voff, nk, st) != hipSuccess) rc = COLA_ERR_HIP;
            fqt[i][k] = vt + voff;             // column-major V is the row-major Q^T
            fq[i][k] = q + voff;
            voff += nk * nk;
        }
        for (auto* d : {&dqt[i], &dq[i]}) {
            std::memset(d, 0, sizeof(*d));
            d->nterms = 1;
            d->nfactors = s.Fv;
            for (int k = 0; k < s.Fv; ++k) d->dims[k] = s.dims[k];
            d->sigma2 = 0.0;
        }
        dqt[i].factors = fqt[i].data();
        dq[i].factors = fq[i].data();
    }
    if (rc == COLA_OK) rc = cola_op_create(dqt.data(), (int32_t)dqt.size(), COLA_PREC_FP64, st, &op->eig_qt);
    if (rc == COLA_OK) rc = cola_op_create(dq.data(), (int32_t)dq.size(), COLA_PREC_FP64, st, &op->eig_q);
    (void)hipStreamSynchronize(st);                        // the operators own copies now
    cleanup();
    if (rc != COLA_OK) {
        if (op->eig_qt) cola_op_destroy(op->eig_qt);
        if (op->eig_q) cola_op_destroy(op->eig_q);
        op->eig_qt = op->eig_q = nullptr;
        dev_free(op, op->eig_lam);
        op->eig_lam = nullptr;
    }
    return rc;
}
}  // namespace

int32_t cola_op_diagonal(cola_op_t op, double* out, void* stream) {
    TraceRange trace_range("cola_op_diagonal");
    if (!op || !out) return COLA_ERR_INVALID_ARG;
    hipStream_t st = S(stream);
    for (const SysInfo& s : op->sys) HIP_TRY(kron_diagonal(diag_args(op, s), out + s.vec_off, false, st));
    return COLA_OK;
}

int32_t cola_diag_estimate(cola_op_t op, const double* Z, int32_t nprobes, int32_t mode, double* out,
                           void* stream) {
    TraceRange trace_range("cola_diag_estimate");
    if (!op || !Z || !out || nprobes < 1) return COLA_ERR_INVALID_ARG;
    if (mode != COLA_DIAG_HUTCHINSON && mode != COLA_DIAG_DOUBLY) return COLA_ERR_INVALID_ARG;
    hipStream_t st = S(stream);
    int32_t rc = ensure_ws(op, nprobes, st);
    if (rc != COLA_OK) return rc;
    double* Q = (double*)op->ws.vq;                  // nprobes * nmax doubles
    const double scale = 1.0 / nprobes;
    int64_t zoff = 0;                                 // doubles of Z consumed by earlier systems
    for (const SysInfo& s : op->sys) {
        double* o = out + s.vec_off;
        if (mode == COLA_DIAG_HUTCHINSON) {
            const double* Zs = Z + (int64_t)nprobes * s.vec_off;
            PassArgs a = base_args(op);
            a.epi = EPI_MATVEC;
            a.Ep = Zs;
            rc = enqueue_mvm(op, s, COLA_PREC_FP64, nprobes, Zs, nullptr, Q, a, st);
            if (rc != COLA_OK) return rc;
            HIP_TRY(probe_accumulate(Zs, Q, s.n, nprobes, scale, o, false, st));
            continue;
        }
        // the diagonal part is exact; every Kronecker term gets its own probes
        DiagArgs da = diag_args(op, s);
        da.J = 0;
        HIP_TRY(kron_diagonal(da, o, false, st));
        for (int j = 0; j < s.J; ++j) {
            SysInfo t = s;                            // term j alone: one term, no diagonal
            t.J = 1;
            for (int k = 0; k < s.Fv; ++k) t.fac_off[k] = s.fac_off[k] + (int64_t)j * s.dims[k] * s.dims[k];
            t.diag_off = -1;
            t.sigma2 = 0.0;
            const double* Zj = Z + zoff + (int64_t)j * nprobes * s.n;
            PassArgs a = base_args(op);
            a.epi = EPI_MATVEC;
            a.Ep = Zj;
            rc = enqueue_mvm(op, t, COLA_PREC_FP64, nprobes, Zj, nullptr, Q, a, st);
            if (rc != COLA_OK) return rc;
            HIP_TRY(probe_accumulate(Zj, Q, s.n, nprobes, scale, o, true, st));
        }
        zoff += (int64_t)s.J * nprobes * s.n;
    }
    return COLA_OK;
}

int32_t cola_eig_solve(cola_op_t op, const double* B, double* X, int32_t nrhs, void* stream) {
    TraceRange trace_range("cola_eig_solve");
    if (!op || !B || !X || nrhs < 1) return COLA_ERR_INVALID_ARG;
    for (const SysInfo& s : op->sys)
        if (s.J != 1 || s.diag_off >= 0) return COLA_ERR_UNSUPPORTED;
    hipStream_t st = S(stream);
    int32_t rc = ensure_eig(op, st);
    if (rc != COLA_OK) return rc;
    rc = ensure_eig_tmp(op, (int64_t)nrhs * op->n_total, st);
    if (rc != COLA_OK) return rc;
    rc = cola_kron_matvec(op->eig_qt, B, op->eig_tmp, nrhs, COLA_F64, COLA_PREC_FP64, stream);
    if (rc != COLA_OK) return rc;
    for (size_t i = 0; i < op->sys.size(); ++i) {
        const SysInfo& s = op->sys[i];
        const double* lam[3] = {nullptr, nullptr, nullptr};
        for (int k = 0; k < s.Fv; ++k) lam[k] = op->eig_lam + op->eig_lam_off[i][k];
        double* y = op->eig_tmp + (int64_t)nrhs * s.vec_off;
        HIP_TRY(eig_scale(y, y, nrhs, s.Fv, s.dims, lam, s.sigma2, st));
    }
    return cola_kron_matvec(op->eig_q, op->eig_tmp, X, nrhs, COLA_F64, COLA_PREC_FP64, stream);
}

int32_t cola_op_memory(cola_op_t op, int64_t* live_bytes, int64_t* peak_bytes, int32_t reset_peak) {
    if (!op) return COLA_ERR_INVALID_ARG;
    int64_t live = (int64_t)op->dev_live, peak = (int64_t)op->dev_peak;
    for (cola_op_s* sub : {op->eig_qt, op->eig_q}) {
        if (!sub) continue;
        int64_t l = 0, p = 0;
        cola_op_memory(sub, &l, &p, reset_peak);
        live += l;
        peak += p;
    }
    if (live_bytes) *live_bytes = live;
    if (peak_bytes) *peak_bytes = peak;
    if (reset_peak) op->dev_peak = op->dev_live;
    return COLA_OK;
}

int32_t cola_op_destroy(cola_op_t op) {
    if (!op) return COLA_OK;
    (void)hipDeviceSynchronize();
    destroy_graphs(op);
    if (op->cap_stream) (void)hipStreamDestroy(op->cap_stream);
    free_resident(op);
    free_ws(op);
    if (op->eig_qt) cola_op_destroy(op->eig_qt);
    if (op->eig_q) cola_op_destroy(op->eig_q);
    for (hipEvent_t e : op->fused_done)
        if (e) (void)hipEventDestroy(e);
    void* ptrs[] = {op->fac64, op->fac32, op->facbf, op->diag64, op->diag32, op->grad_buf, op->eig_lam,
                    op->eig_tmp, op->fused_slots, op->slq_buf, op->pc_dinv, op->small_sys};
    for (void* p : ptrs)
        if (p) dev_free(op, p);
    delete op;
    return COLA_OK;
}

int32_t cola_op_size(cola_op_t op, int64_t* n_total, int32_t* nsys) {
    if (!op) return COLA_ERR_INVALID_ARG;
    if (n_total) *n_total = op->n_total;
    if (nsys) *nsys = (int32_t)op->sys.size();
    return COLA_OK;
}

int32_t cola_kron_matvec(cola_op_t op, const void* X, void* Y, int32_t nrhs, int32_t dtype, int32_t prec,
                         void* stream) {
    TraceRange trace_range("cola_kron_matvec");
    if (!op || !X || !Y || nrhs < 1) return COLA_ERR_INVALID_ARG;
    if (prec == COLA_PREC_FP64) {
        if (dtype != COLA_F64) return COLA_ERR_INVALID_ARG;
    } else {
        if (prec != op->prec || dtype != COLA_F32) return COLA_ERR_INVALID_ARG;
    }
    hipStream_t st = S(stream);
    int32_t rc = ensure_ws(op, nrhs, st);
    if (rc != COLA_OK) return rc;
    const size_t esz = (dtype == COLA_F64) ? 8 : 4;
    for (const SysInfo& s : op->sys) {
        const char* xs = (const char*)X + esz * (size_t)nrhs * s.vec_off;
        char* ys = (char*)Y + esz * (size_t)nrhs * s.vec_off;
        PassArgs a = base_args(op);
        a.epi = EPI_MATVEC;
        a.Ep = xs;
        rc = enqueue_mvm(op, s, prec, nrhs, xs, nullptr, ys, a, st);
        if (rc != COLA_OK) return rc;
    }
    return COLA_OK;
}

int32_t cola_kron_matvec_noalloc(cola_op_t op, const void* X, void* Y, int32_t nrhs, int32_t dtype, int32_t prec,
                                 void* stream) {
    TraceRange trace_range("cola_kron_matvec_noalloc");
    if (!op || !X || !Y || nrhs < 1) return COLA_ERR_INVALID_ARG;
    if (prec == COLA_PREC_FP64) {
        if (dtype != COLA_F64) return COLA_ERR_INVALID_ARG;
    } else {
        if (prec != op->prec || dtype != COLA_F32) return COLA_ERR_INVALID_ARG;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return COLA_ERR_HIP;
    if (dev != op->device) return COLA_ERR_INVALID_ARG;
    const size_t esz = (dtype == COLA_F64) ? 8 : 4;
    const size_t half = kScratchBytes / 2;
    // each intermediate holds at most Jmax * nrhs * nmax elements of the working precision
    if ((double)op->Jmax * (double)nrhs * (double)op->nmax * (double)esz > (double)half) return COLA_ERR_SCRATCH;
    void* base = nullptr;
    int32_t rc = scratch_address(dev, &base);
    if (rc != COLA_OK) return rc;
    void* const inter[2] = {base, (char*)base + half};
    hipStream_t st = S(stream);
    for (const SysInfo& s : op->sys) {
        const char* xs = (const char*)X + esz * (size_t)nrhs * s.vec_off;
        char* ys = (char*)Y + esz * (size_t)nrhs * s.vec_off;
        PassArgs a;
        std::memset(&a, 0, sizeof(a));                  // a product needs no reduction buffers
        a.epi = EPI_MATVEC;
        a.Ep = xs;
        rc = enqueue_mvm(op, s, prec, nrhs, xs, nullptr, ys, a, st, inter, nullptr);
        if (rc != COLA_OK) return rc;
    }
    return COLA_OK;
}

int32_t cola_cg_solve(cola_op_t op, const double* B, double* X, int32_t nrhs, const cola_solve_opts* opts,
                      cola_solve_info* info, void* stream) {
    TraceRange trace_range("cola_cg_solve");
    if (!op || !B || !X || nrhs < 1) return COLA_ERR_INVALID_ARG;
    int32_t rc = check_opts(op, opts);
    if (rc != COLA_OK) return rc;
    hipStream_t st = S(stream);
    const bool want_hist = opts->hist != nullptr;
    if (want_hist)
        HIP_TRY(fill_f64(opts->hist, __builtin_nan(""), (int64_t)op->sys.size() * nrhs * opts->hist_len, st));
    if (op->resident_ok && op->use_resident && opts->prec == COLA_PREC_FP32 &&
        opts->refine == COLA_REFINE_RELIABLE && !opts->x0_given && !want_hist)
        return solve_resident(op, B, X, nrhs, opts, info, st);
    if (op->small_ok && op->use_small && opts->prec == COLA_PREC_FP64 && opts->precond == COLA_PRECOND_NONE)
        return solve_small(op, B, X, nrhs, opts, info, st);
    rc = ensure_ws(op, nrhs, st);
    if (rc != COLA_OK) return rc;
    // restarted refinement's inner solves each start over on a normalised residual: no history
    const bool record = want_hist && !(opts->prec != COLA_PREC_FP64 && opts->refine == COLA_REFINE_RESTART);
    for (size_t i = 0; i < op->sys.size(); ++i) {
        const SysInfo& s = op->sys[i];
        const size_t off = (size_t)nrhs * s.vec_off;
        op->ws.rh = ResHist{};
        if (record) {
            op->ws.rh.data = opts->hist + i * (size_t)nrhs * opts->hist_len;
            op->ws.rh.stride = opts->hist_stride;
            op->ws.rh.len = opts->hist_len;
        }
        rc = solve_system(op, s, B + off, X + off, nrhs, opts, info ? info + i * nrhs : nullptr, st);
        op->ws.rh = ResHist{};
        if (rc != COLA_OK) return rc;
    }
    return COLA_OK;
}

int32_t cola_slq_logdet(cola_op_t op, const double* Z, int32_t nprobes, double tol, int32_t max_iters,
                        double* X, double* logdet, double* est, cola_solve_info* info, void* stream) {
    TraceRange trace_range("cola_slq_logdet");
    if (!op || !Z || !logdet || nprobes < 1 || !finite_pos(tol) || max_iters < 1) return COLA_ERR_INVALID_ARG;
    if (max_iters > kSlqMaxSteps) return COLA_ERR_INVALID_ARG;
    hipStream_t st = S(stream);
    int32_t rc = ensure_ws(op, nprobes, st);
    if (rc != COLA_OK) return rc;
    const size_t hist_elems = (size_t)nprobes * 2 * (size_t)max_iters;
    const size_t need = hist_elems + (size_t)nprobes;              // history, then per-probe estimates
    if (op->slq_elems < need) {
        if (op->slq_buf) dev_free(op, op->slq_buf);
        op->slq_buf = nullptr;
        op->slq_elems = 0;
        rc = dev_alloc(op, (void**)&op->slq_buf, need * sizeof(double));
        if (rc != COLA_OK) return rc;
        op->slq_elems = need;
    }
    cola_solve_opts o{};
    o.tol = tol;
    o.max_iters = max_iters;
    o.prec = COLA_PREC_FP64;
    o.check_every = 32;
    Workspace& w = op->ws;
    for (size_t i = 0; i < op->sys.size(); ++i) {
        const SysInfo& s = op->sys[i];
        const size_t off = (size_t)nprobes * s.vec_off;
        w.hist = op->slq_buf;
        w.hist_len = max_iters;
        rc = solve_system(op, s, Z + off, X ? X + off : nullptr, nprobes, &o, info ? info + i * nprobes : nullptr, st);
        w.hist = nullptr;
        w.hist_len = 0;
        if (rc != COLA_OK) return rc;
        double* e = est ? est + i * nprobes : op->slq_buf + hist_elems;
        HIP_TRY(slq_logdet(op->slq_buf, max_iters, w.cg, nprobes, e, logdet + i, st));
    }
    return COLA_OK;
}

int32_t cola_cg_solve_backward(cola_op_t op, const double* X, const double* G, int32_t nrhs,
                               const cola_solve_opts* opts, double* Lambda, void* const* dfactors,
                               void* const* ddiag, double* dsigma2, cola_solve_info* info, void* stream) {
    TraceRange trace_range("cola_cg_solve_backward");
    if (!op || !X || !G || !Lambda || nrhs < 1) return COLA_ERR_INVALID_ARG;
    int32_t rc = cola_cg_solve(op, G, Lambda, nrhs, opts, info, stream);
    if (rc != COLA_OK) return rc;
    hipStream_t st = S(stream);
    // the factor contractions stage through the solve workspace, which the one-workgroup
    // and resident solve paths do not size for nrhs right-hand sides
    rc = ensure_ws(op, nrhs, st);
    if (rc != COLA_OK) return rc;
    for (size_t i = 0; i < op->sys.size(); ++i) {
        const SysInfo& s = op->sys[i];
        const size_t off = (size_t)nrhs * s.vec_off;
        rc = grad_system(op, s, X + off, Lambda + off, nrhs, dfactors ? dfactors + s.grad_off : nullptr,
                         ddiag ? ddiag[i] : nullptr, dsigma2 ? dsigma2 + i : nullptr, st);
        if (rc != COLA_OK) return rc;
    }
    return COLA_OK;
}

int32_t cola_logdet_grad(cola_op_t op, const double* Z, int32_t nprobes, const cola_solve_opts* opts,
                         double* Lambda, void* const* dfactors, void* const* ddiag, double* dsigma2,
                         cola_solve_info* info, void* stream) {
    TraceRange trace_range("cola_logdet_grad");
    if (!op || !Z || !Lambda || nprobes < 1) return COLA_ERR_INVALID_ARG;
    int32_t rc = cola_cg_solve(op, Z, Lambda, nprobes, opts, info, stream);      // Lambda = A^{-1} Z
    if (rc != COLA_OK) return rc;
    hipStream_t st = S(stream);
    rc = ensure_ws(op, nprobes, st);
    if (rc != COLA_OK) return rc;
    const double scale = -1.0 / nprobes;        // the solve VJP's sign and the mean over probes
    for (size_t i = 0; i < op->sys.size(); ++i) {
        const SysInfo& s = op->sys[i];
        const size_t off = (size_t)nprobes * s.vec_off;
        rc = grad_system(op, s, Z + off, Lambda + off, nprobes, dfactors ? dfactors + s.grad_off : nullptr,
                         ddiag ? ddiag[i] : nullptr, dsigma2 ? dsigma2 + i : nullptr, st, scale);
        if (rc != COLA_OK) return rc;
    }
    return COLA_OK;
}

int32_t cola_trace_enable(int32_t enable) {
    g_trace_on.store(enable != 0 ? 1 : 0, std::memory_order_relaxed);
    return COLA_OK;
}

int32_t cola_op_set_engine(cola_op_t op, int32_t engine, int32_t enable) {
    if (!op) return COLA_ERR_INVALID_ARG;
    const bool on = enable != 0;
    switch (engine) {
        case COLA_ENGINE_FUSED_CG: op->use_fused = on; break;
        case COLA_ENGINE_GEMM2: op->use_gemm2 = on; break;
        case COLA_ENGINE_GEMM3: op->use_gemm3 = on; break;
        case COLA_ENGINE_SLAB: op->use_slab = on; break;
        case COLA_ENGINE_RESIDENT: op->use_resident = on; break;
        case COLA_ENGINE_SMALL64: op->use_small = on; break;
        case COLA_ENGINE_GEMM64: op->use_gemm64 = on; break;
        default: return COLA_ERR_INVALID_ARG;
    }
    (void)hipDeviceSynchronize();
    destroy_graphs(op);              // captured chunks embed the previous choice
    return COLA_OK;
}

int32_t cola_autotune(cola_op_t op, int32_t nrhs, void* stream) {
    TraceRange trace_range("cola_autotune");
    if (!op || nrhs < 1) return COLA_ERR_INVALID_ARG;
    return autotune_op(op, nrhs, S(stream));
}

// The device line of an exported tile table: architecture name and compute-unit count.
static std::string tile_device_tag() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown 0";
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    return arch + " " + std::to_string(prop.multiProcessorCount);
}

int32_t cola_autotune_export(cola_op_t op, char* buf, int64_t cap, int64_t* len) {
    if (!op || !len || (buf && cap < 1)) return COLA_ERR_INVALID_ARG;
    std::string s = "device " + tile_device_tag() + "\n";
    for (const auto& kv : op->tiles) {
        const PassKey& k = kv.first;
        s += std::to_string(k.prec) + " " + std::to_string(k.rows) + " " + std::to_string(k.nk) + " " +
             std::to_string(k.B) + " " + std::to_string(k.g) + " " + std::to_string(kv.second.wm) + " " +
             std::to_string(kv.second.wn) + "\n";
    }
    *len = (int64_t)s.size();
    if (!buf) return COLA_OK;
    if ((int64_t)s.size() + 1 > cap) return COLA_ERR_INVALID_ARG;
    std::memcpy(buf, s.c_str(), s.size() + 1);
    return COLA_OK;
}

int32_t cola_autotune_import(cola_op_t op, const char* text) {
    if (!op || !text) return COLA_ERR_INVALID_ARG;
    const std::string here = tile_device_tag();
    std::map<PassKey, TileCfg> got;
    bool for_here = false;
    const char* p = text;
    while (*p) {
        const char* e = std::strchr(p, '\n');
        const std::string line(p, e ? (size_t)(e - p) : std::strlen(p));
        p = e ? e + 1 : p + line.size();
        if (line.empty()) continue;
        if (line.compare(0, 7, "device ") == 0) {
            for_here = line.substr(7) == here;
            continue;
        }
        long long v[7];
        int used = 0;
        if (std::sscanf(line.c_str(), "%lld %lld %lld %lld %lld %lld %lld%n", &v[0], &v[1], &v[2], &v[3], &v[4],
                        &v[5], &v[6], &used) != 7 || line.find_first_not_of(" \t\r", (size_t)used) != std::string::npos)
            return COLA_ERR_INVALID_ARG;
        const bool cfg_ok = (v[5] == 1 || v[5] == 2 || v[5] == 4) && (v[6] == 1 || v[6] == 2 || v[6] == 4);
        const bool key_ok = v[0] >= COLA_PREC_FP64 && v[0] <= COLA_PREC_BF16X3 && (v[1] == 0 || v[1] == 1) &&
                            v[2] >= 1 && v[3] >= 1 && v[4] >= 1;
        if (!cfg_ok || !key_ok) return COLA_ERR_INVALID_ARG;
        if (!for_here) continue;                         // tuned on another device: not used here
        got[PassKey{(int)v[0], (int)v[1], (int64_t)v[2], (int64_t)v[3], (int64_t)v[4]}] =
            TileCfg{(int)v[5], (int)v[6]};
    }
    if (got.empty()) return COLA_OK;
    (void)hipDeviceSynchronize();
    for (const auto& kv : got) op->tiles[kv.first] = kv.second;
    destroy_graphs(op);                                  // captured chunks embed the previous tiles
    op->tiles_version += 1;
    return COLA_OK;
}

int32_t cola_profile_enable(cola_op_t op, int32_t enable) {
    if (!op) return COLA_ERR_INVALID_ARG;
    (void)hipDeviceSynchronize();
    op->prof.clear();
    op->prof.enabled = enable != 0;
    return COLA_OK;
}

int32_t cola_profile_read(cola_op_t op, const char* kernel, double* total_ms, int64_t* launches) {
    if (!op || !kernel || !total_ms || !launches) return COLA_ERR_INVALID_ARG;
    if (hipDeviceSynchronize() != hipSuccess) return COLA_ERR_HIP;
    op->prof.read(kernel, total_ms, launches);
    return COLA_OK;
}

}  // extern "C"

// ===========================================================================
namespace cola {

std::atomic<int> g_trace_on{0};

TraceRange::TraceRange(const char* name) : on(g_trace_on.load(std::memory_order_relaxed) != 0) {
    if (on) roctxRangePushA(name);
}

TraceRange::~TraceRange() {
    if (on) roctxRangePop();
}

int32_t ensure_workspace(cola_op_s* op, int nrhs, hipStream_t st) { return ensure_ws(op, nrhs, st); }

hipEvent_t Profiler::get() {
    if (!pool_.empty()) {
        hipEvent_t e = pool_.back();
        pool_.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// Inside a stream capture an event is recorded as an external event-record
// node (a plain record would only become a dependency edge of the graph).
static void record_event(hipEvent_t e, hipStream_t s, bool capturing) {
    if (capturing) (void)hipEventRecordWithFlags(e, s, hipEventRecordExternal);
    else (void)hipEventRecord(e, s);
}

void Profiler::begin(const char* name, hipStream_t s) {
    hipEvent_t e = capture_list ? nullptr : get();
    if (capture_list) (void)hipEventCreate(&e);       // owned by the graph being captured
    record_event(e, s, capture_list != nullptr);
    pending_[name] = e;
}

void Profiler::end(const char* name, hipStream_t s) {
    auto it = pending_.find(name);
    if (it == pending_.end()) return;
    hipEvent_t e = nullptr;
    if (capture_list) (void)hipEventCreate(&e);
    else e = get();
    record_event(e, s, capture_list != nullptr);
    ProfPair pr{name, it->second, e};
    if (capture_list) capture_list->push_back(pr);
    else open_.push_back(pr);
    pending_.erase(it);
}

void Profiler::harvest(const std::vector<ProfPair>& pairs) {
    for (const ProfPair& pr : pairs) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, pr.a, pr.b) == hipSuccess) {
            auto& tot = totals_[pr.name];
            tot.first += t;
            tot.second += 1;
        } else {
            (void)hipGetLastError();
        }
    }
}

void Profiler::read(const std::string& name, double* ms, int64_t* launches) {
    harvest(open_);
    for (auto& pr : open_) {
        pool_.push_back(pr.a);
        pool_.push_back(pr.b);
    }
    open_.clear();
    auto it = totals_.find(name);
    *ms = it == totals_.end() ? 0.0 : it->second.first;
    *launches = it == totals_.end() ? 0 : it->second.second;
}

void Profiler::clear() {
    for (auto& pr : open_) {
        pool_.push_back(pr.a);
        pool_.push_back(pr.b);
    }
    open_.clear();
    for (auto& kv : pending_) pool_.push_back(kv.second);
    pending_.clear();
    totals_.clear();
}

Profiler::~Profiler() {
    clear();
    for (hipEvent_t e : pool_) (void)hipEventDestroy(e);
}

}  // namespace cola
