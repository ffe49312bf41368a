// Operator handle and workspace (host side of libcola).
#pragma once
#include <array>
#include <map>
#include <tuple>
#include <string>
#include <utility>
#include <vector>

#include "common.h"
#include "contract.h"

namespace cola {

// One independent system, with the Kronecker structure made at least two
// modes deep (a single dense factor K becomes [1] (x) K).
struct SysInfo {
    int J = 1;             // terms
    int F = 2;             // factors as given (1..3)
    int Fv = 2;            // modes used by the passes (max(F, 2))
    int64_t dims[3] = {1, 1, 1};
    int64_t n = 1;
    int64_t fac_off[3] = {0, 0, 0};   // mode k: term t's factor at fac_off[k] + t*dims[k]^2
    int64_t diag_off = -1;            // offset in the diagonal buffers, -1: none
    double sigma2 = 0.0;
    int64_t vec_off = 0;              // unknowns of all earlier systems
    int64_t grad_off = 0;             // this system's first entry in a dfactors pointer list
};

struct Workspace {
    int nrhs = 0;
    int64_t part_stride = 0;
    void* vx = nullptr; void* vr = nullptr; void* vp = nullptr; void* vq = nullptr;  // CG vectors (8 B / elem)
    void* inter[2] = {nullptr, nullptr};                                             // MVM intermediates
    double* r64 = nullptr;                                                            // FP64 residual
    double* x64 = nullptr;                                                            // FP64 solution
    double* b64 = nullptr;                                                            // FP64 right-hand sides
    double* partials = nullptr;
    uint32_t* counters = nullptr;
    CgState* cg = nullptr;
    OuterState* outer = nullptr;
    SolveCounters* cnt = nullptr;
    int32_t* host_flag = nullptr;     // pinned
    double* hist = nullptr;           // while set: (alpha, beta) of every FP64 CG iteration, hist_len per RHS
    int hist_len = 0;
    ResHist rh;                       // while set: residual history of the current solve (its system's rows)
};

// Per-kernel-class timing with HIP events recorded around launches.  Direct
// launches keep their event pairs until read; launches captured into a
// graph record into that graph's own event list, which is harvested after
// every replay (a replay overwrites the events of the previous one).
struct ProfPair { std::string name; hipEvent_t a, b; };

class Profiler {
public:
    bool enabled = false;
    std::vector<ProfPair>* capture_list = nullptr;   // set while capturing a graph
    void begin(const char* name, hipStream_t s);
    void end(const char* name, hipStream_t s);
    void harvest(const std::vector<ProfPair>& pairs);
    void clear();
    void read(const std::string& name, double* ms, int64_t* launches);
    hipEvent_t get();
    ~Profiler();
private:
    std::vector<hipEvent_t> pool_;
    std::vector<ProfPair> open_;
    std::map<std::string, hipEvent_t> pending_;
    std::map<std::string, std::pair<double, int64_t>> totals_;
};

// A captured chunk of CG iterations, replayed with hipGraphLaunch.
struct ChunkGraph {
    hipGraphExec_t exec = nullptr;
    std::vector<ProfPair> ev;       // profiling events inside the graph
};
struct GraphSet {
    ChunkGraph g[2];                // alternated so one chunk runs while the host polls the other
    hipEvent_t done[2] = {nullptr, nullptr};
};
struct GraphKey {
    const void* sys; int prec; int nrhs; const void* x; const void* r; const void* p; const void* q;
    int chunk; int profiled; int tiles_version; const void* hist; const void* rhist; int rstride; int rlen;
    bool operator<(const GraphKey& o) const {
        return std::tie(sys, prec, nrhs, x, r, p, q, chunk, profiled, tiles_version, hist, rhist, rstride, rlen) <
               std::tie(o.sys, o.prec, o.nrhs, o.x, o.r, o.p, o.q, o.chunk, o.profiled, o.tiles_version, o.hist,
                        o.rhist, o.rstride, o.rlen);
    }
};

// Key of a contraction pass for the tile table: (prec, rows, nk, B, G-per-rhs).
struct PassKey {
    int prec; int rows; int64_t nk; int64_t B; int64_t g;
    bool operator<(const PassKey& o) const {
        if (prec != o.prec) return prec < o.prec;
        if (rows != o.rows) return rows < o.rows;
        if (nk != o.nk) return nk < o.nk;
        if (B != o.B) return B < o.B;
        return g < o.g;
    }
};

}  // namespace cola

struct cola_op_s {
    int device = 0;
    int prec = COLA_PREC_FP64;
    std::vector<cola::SysInfo> sys;
    int64_t n_total = 0, nmax = 0;
    int Jmax = 1;
    int64_t fac_elems = 0, diag_elems = 0;
    double* fac64 = nullptr;
    float* fac32 = nullptr;
    __bf16* facbf = nullptr;        // nsplit planes of fac_elems
    int nsplit = 0;
    double* diag64 = nullptr;
    float* diag32 = nullptr;
    cola::Workspace ws;
    cola::Profiler prof;
    std::map<cola::PassKey, cola::TileCfg> tiles;
    double* grad_buf = nullptr;     // split-K slices of factor gradients that exceed the workspace
    size_t grad_buf_elems = 0;
    int tiles_version = 0;          // bumped when the tile table changes (invalidates graphs)
    bool graphs_ok = true;          // false after a capture failure: launch directly
    bool use_slab = true;           // fuse modes 2 and 3 of three-mode terms when slabs fit in LDS
    bool use_gemm2 = true;          // BF16 two-mode operators with large modes: dense-GEMM MVM
    bool use_gemm3 = true;          // FP32 one-term three-mode operators with 256-wide modes: dense-GEMM MVM
    bool use_gemm64 = true;         // FP64 passes of two-mode operators with modes multiples of 256: dense FP64 GEMMs
    bool use_fused = true;          // FP32 one-term three-mode operators with 64-wide modes: persistent fused CG
    int fused_max_blocks = -1;      // co-resident fused-CG blocks (-1: not yet queried)
    double* slq_buf = nullptr;      // SLQ: CG coefficient history and per-probe estimates
    size_t slq_elems = 0;
    double* fused_slots = nullptr;      // fused-CG barrier slots (3 * fused_max_blocks), then the time-out flag
    hipEvent_t fused_done[2] = {nullptr, nullptr};
    bool resident_ok = false;       // every system fits the resident batched kernel
    bool small_ok = false;          // every system fits the one-workgroup FP64 kernel
    bool use_small = true;
    void* small_sys = nullptr;      // ResSys[nsys] of the one-workgroup FP64 kernel
    bool use_resident = true;
    int num_cus = 0;
    // resident-path workspace (allocated for res_nrhs right-hand sides)
    int res_nrhs = 0;
    void* res_sys = nullptr;        // ResSys[nsys]
    int32_t* res_order = nullptr;   // nsys * nrhs items, largest systems first
    float* res_x = nullptr; float* res_r = nullptr; float* res_p = nullptr;
    double* res_t64 = nullptr;
    cola::CgState* res_st = nullptr;
    uint32_t* res_queue = nullptr;
    hipStream_t cap_stream = nullptr;
    std::map<cola::GraphKey, cola::GraphSet> graphs;
    // Kronecker-eigen solve: operators of the eigenvector factors Q^T and Q
    // (one term per system, FP64), eigenvalues per system and mode, scratch
    cola_op_s* eig_qt = nullptr;
    cola_op_s* eig_q = nullptr;
    double* eig_lam = nullptr;
    std::vector<std::array<int64_t, 3>> eig_lam_off;
    double* eig_tmp = nullptr;
    int64_t eig_tmp_elems = 0;
    // preconditioned CG: Jacobi inverse diagonal (n_total, packed by system) and the
    // Kronecker-eigen preconditioner's shift per system
    double* pc_dinv = nullptr;
    std::vector<double> pc_shift;
    // device memory held by this op's own allocations (bytes), and its high-water mark
    std::map<void*, size_t> dev_sizes;
    size_t dev_live = 0, dev_peak = 0;
};

namespace cola {
// Allocate (or keep) the per-op workspace for nrhs right-hand sides.
int32_t ensure_workspace(cola_op_s* op, int nrhs, hipStream_t st);
// Device allocations owned by op, counted in its live and peak bytes
// (dev_alloc returns COLA_ERR_OOM and sets *p = nullptr on failure).
int32_t dev_alloc(cola_op_s* op, void** p, size_t bytes);
void dev_free(cola_op_s* op, void* p);
}
