/*
 * cola.h - C ABI of the MI355X (gfx950) sum-of-Kronecker conjugate-gradient library.
 *
 * Operator (CoLA, arxiv 2309.03060; Sec. 3.1 base operators Dense and Diagonal,
 * Sec. 3.2 Sum and Kronecker compositions, Table 2 Kronecker MVM cost):
 *
 *     A = sum_{j<J} ( K_j1 (x) K_j2 [(x) K_j3] ) + diag(d) + sigma2 * I
 *
 * A is assumed symmetric positive definite, so solves use conjugate gradients
 * (the PSD base case, Sec. 3.2 "Decoration/annotation operators" and App. C's
 * table of base-case iterative methods).  Gradients follow the solve VJP of
 * App. B.2 (autograd rule 1).
 *
 * Conventions used by every entry point
 * -------------------------------------
 *  - vec is row-major: the element of multi-index (i1, i2, i3) sits at
 *    i1*n2*n3 + i2*n3 + i3, so (K1 (x) K2) x = vec(K1 X K2^T), X = x as n1 x n2.
 *  - Factors are dense, row-major n_k x n_k, float64, in device memory.
 *  - Vectors are packed: system s (n_s unknowns) with nrhs right-hand sides
 *    occupies nrhs * n_s consecutive elements, right-hand side r of it at
 *    offset r * n_s; systems follow each other in the order given at create.
 *  - All device pointers must be 16-byte aligned and refer to memory on the
 *    device that is current when the call is made.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue work on
 *    it and return; outputs are valid once the stream has reached that point.
 *    The solve entry points may also wait on the stream to poll convergence
 *    (see cola_solve_opts.check_every).
 *  - Return value: COLA_OK, or a negative error for invalid arguments, an
 *    allocation failure or a HIP error.  Numerical outcomes (non-convergence,
 *    breakdown, non-finite data) are reported per right-hand side in
 *    cola_solve_info, not as the return value.
 *  - Errors leave caller buffers in an unspecified state but never free or
 *    retain them.  The library keeps no pointer to caller memory past a call.
 *  - Thread safety: one op may be used by one host thread / stream at a time.
 */
#ifndef COLA_H
#define COLA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes ---------------------------------------------------------- */
#define COLA_OK                 0
#define COLA_NOT_CONVERGED      1   /* max_iters / max_sweeps reached; x is the last iterate */
#define COLA_STAGNATED          2   /* refinement stopped halving the residual twice in a row */
#define COLA_ERR_INVALID_ARG  (-1)
#define COLA_ERR_NOT_SPD      (-2)  /* CG breakdown: p^T A p <= 0 */
#define COLA_ERR_NONFINITE    (-3)  /* NaN / Inf met in b or during the iteration */
#define COLA_ERR_OOM          (-4)
#define COLA_ERR_HIP          (-5)
#define COLA_ERR_UNSUPPORTED  (-6)
#define COLA_ERR_SCRATCH      (-7)  /* call too large for cola_kron_matvec_noalloc's static scratch */

/* element types of caller vectors --------------------------------------- */
#define COLA_F64 0
#define COLA_F32 1

/* working precision of the Kronecker MVM and of the inner CG vectors ----- */
#define COLA_PREC_FP64   0   /* FP64 factors, FP64 MFMA, FP64 vectors             */
#define COLA_PREC_FP32   1   /* FP32 factors, FP32 MFMA, FP32 vectors             */
#define COLA_PREC_BF16   2   /* BF16 factors and operands, FP32 accumulation      */
#define COLA_PREC_BF16X3 3   /* 3-way BF16 split of factors and operands (~FP32)  */

typedef struct cola_op_s* cola_op_t;

/* One independent SPD system.  `factors` is a HOST array of nterms*nfactors
 * DEVICE pointers: factor k of term j at index j*nfactors + k, each n_k x n_k
 * float64 row-major.  Every term has the same dims.  `diag` is a device
 * pointer to n float64 values or NULL (no diagonal term besides sigma2). */
typedef struct {
    int32_t nterms;              /* J >= 1                          */
    int32_t nfactors;            /* F in {1, 2, 3}                  */
    int64_t dims[3];             /* n_1..n_F >= 1; unused entries ignored */
    const void* const* factors;  /* host array of device pointers   */
    const void* diag;            /* device pointer or NULL          */
    double sigma2;               /* >= 0, finite                    */
} cola_system_desc;

/* Build an operator from nsys systems (Sec. 3.2: the Sum of Kronecker terms
 * and the Diagonal is represented by its parts, never formed densely).
 * The library copies the factors and diagonal into its own FP64 master copy
 * and converts a working copy in precision `prec` (COLA_PREC_*).  Copies
 * are enqueued on `stream`; the caller may free its buffers once the stream
 * has passed this call.  On success *out receives the handle. */
int32_t cola_op_create(const cola_system_desc* systems, int32_t nsys, int32_t prec,
                       void* stream, cola_op_t* out);

/* Release the operator and every device buffer it owns (synchronises the
 * device first).  NULL is accepted. */
int32_t cola_op_destroy(cola_op_t op);

/* Device memory held by the operator (App. B.2: the adjoint rules keep the
 * backward pass's memory independent of the number of solver iterations;
 * this is how that is measured).  *live_bytes: bytes of every device buffer
 * the operator and its internal sub-operators own right now (factor copies,
 * CG workspace, gradient and log-det buffers); *peak_bytes: the largest value
 * live_bytes has reached since creation or the last reset (summed over the
 * sub-operators, so an upper bound when they peaked at different times).
 * Either pointer may be NULL; reset_peak != 0 sets the peak to the current
 * live bytes after reading it.  Host-side bookkeeping only: no device call. */
int32_t cola_op_memory(cola_op_t op, int64_t* live_bytes, int64_t* peak_bytes, int32_t reset_peak);

/* Total unknowns summed over systems (n_total) and number of systems. */
int32_t cola_op_size(cola_op_t op, int64_t* n_total, int32_t* nsys);

/* Y = A X (Sec. 3.2: MVM of the Sum = sum of the children's MVMs; each
 * Kronecker term applied mode by mode at the Table 2 cost).  X and Y are
 * packed vectors of nrhs right-hand sides, element type `dtype`:
 *   prec == COLA_PREC_FP64            requires dtype == COLA_F64;
 *   prec == the op's working precision requires dtype == COLA_F32.
 * X and Y must not overlap. */
int32_t cola_kron_matvec(cola_op_t op, const void* X, void* Y, int32_t nrhs,
                         int32_t dtype, int32_t prec, void* stream);

/* Y = A X exactly as cola_kron_matvec, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  The pass intermediates live in a static device array
 * of 64 MiB inside the library (two halves of 32 MiB) instead of the op's
 * workspace, so the call allocates nothing (no hipMalloc, no workspace growth,
 * no profiling events) and enqueues only kernels on `stream`.
 *   Limit: (largest term count) * nrhs * (largest system's n) * (8 for
 *   COLA_PREC_FP64, else 4) bytes must not exceed 32 MiB; larger calls return
 *   COLA_ERR_SCRATCH and enqueue nothing.
 *   The device that is current must be the op's device (else
 *   COLA_ERR_INVALID_ARG).  Its first call on a device looks up that device's
 *   copy of the array once (hipGetSymbolAddress).
 *   Every call on one GPU shares that GPU's array, which keeps the last call's
 *   contents (no call needs it cleared): calls that overlap on one GPU - two
 *   streams, or two host threads - race and must be serialised by the caller.
 * Arguments, layout and the other errors are those of cola_kron_matvec. */
int32_t cola_kron_matvec_noalloc(cola_op_t op, const void* X, void* Y, int32_t nrhs, int32_t dtype,
                                 int32_t prec, void* stream);

/* mixed-precision scheme (cola_solve_opts.refine) ------------------------ */
#define COLA_REFINE_RELIABLE 0  /* one low-precision CG; its residual is replaced by the FP64 true
                                   residual whenever it has dropped by inner_tol (reliable updates) */
#define COLA_REFINE_RESTART  1  /* classical refinement: restarted inner CG solves to inner_tol,
                                   FP64 residual between sweeps (at most max_sweeps sweeps)        */

/* preconditioner (cola_solve_opts.precond; FP64 solves only) ------------- */
#define COLA_PRECOND_NONE     0  /* plain CG */
#define COLA_PRECOND_JACOBI   1  /* M = Diag(A), exact by the Sum and Kronecker diagonal rules (App. A) */
#define COLA_PRECOND_KRON_EIG 2  /* M = (first Kronecker term) + c I with c = Tr(A - first term) / n,
                                    applied exactly by the Kronecker eigen rules (App. A); for one term
                                    plus sigma2 I, M = A and CG ends after one step */

/* Solve options. */
typedef struct {
    double  tol;          /* target relative residual ||b - A x|| / ||b|| per RHS, > 0 */
    int32_t max_iters;    /* max CG iterations per (inner) solve, >= 1                  */
    int32_t prec;         /* COLA_PREC_FP64, or the op's working precision              */
    double  inner_tol;    /* in (0, 1): residual reduction between reliable updates, or the
                             relative residual target of each restarted inner solve.  A
                             small reduction lets the low-precision recurrence drift far
                             from the true residual before its first replacement: on a
                             kappa ~ 1e7 operator 0.01 diverged where 0.1 to 0.9 converged
                             (0.3 to 0.9 in the fewest iterations)                          */
    int32_t max_sweeps;   /* restarted refinement: sweeps (>= 1); otherwise ignored       */
    int32_t check_every;  /* >0: the host waits on the stream every this many CG
                             iterations to stop early once all RHS converged;
                             0: never wait - all work is enqueued (max_iters
                             iterations per sweep, device-side early exit), which
                             makes the call safe under stream capture           */
    int32_t refine;       /* COLA_REFINE_RELIABLE or COLA_REFINE_RESTART (prec != FP64) */
    int32_t precond;      /* COLA_PRECOND_*; anything but NONE needs prec == COLA_PREC_FP64
                             (else COLA_ERR_UNSUPPORTED).  Preconditioned CG takes the
                             textbook recurrence (z = M^{-1} r, beta = r.z / r_old.z_old,
                             p = z + beta p) and stops on ||b - A x|| <= tol ||b|| as
                             plain CG does; the first call sets M up (Jacobi: one pass
                             over the diagonal rules; Kronecker-eigen: the first term's
                             factor eigendecompositions, waiting on the stream). */
    int32_t x0_given;     /* 0: x0 = 0.  != 0: X holds the initial iterate on entry (warm
                             start, e.g. resuming a solve stopped by max_iters from its X):
                             CG starts from r0 = b - A x0 formed with the FP64 factors, and
                             tolerances stay relative to ||b||                          */
    int32_t hist_stride;  /* > 0 with hist: record the recursive relative residual
                             ||r_k|| / ||b|| after every hist_stride-th iteration (the
                             residual against MVM count of the paper's convergence plots) */
    int32_t hist_len;     /* entries per right-hand side in hist                          */
    int32_t reserved;
    double* hist;         /* NULL, or DEVICE nsys*nrhs*hist_len doubles, row (system, RHS)
                             in packing order, entry k after iteration (k+1)*hist_stride;
                             the call first fills every entry with NaN.  Mixed precision
                             records the working-precision recurrence (reset to the FP64
                             residual at each reliable update); restarted refinement
                             records nothing                                              */
} cola_solve_opts;

/* Per (system, RHS) outcome, written to DEVICE memory in stream order. */
typedef struct {
    int32_t status;       /* COLA_OK, COLA_NOT_CONVERGED, COLA_STAGNATED,
                             COLA_ERR_NOT_SPD or COLA_ERR_NONFINITE            */
    int32_t iters;        /* CG iterations summed over all sweeps               */
    int32_t sweeps;       /* refinement sweeps or reliable updates (0 for a plain solve) */
    int32_t reserved;
    double  relres_recursive; /* ||r|| / ||b|| of the CG recurrence at its end (restarted
                                 refinement: its FP64 residual)                        */
    double  relres_true;  /* ||b - A x|| / ||b|| of the returned x with the FP64 factors
                             (absolute residuals for b = 0).  Plain FP64 solves stop on
                             the recursive residual; mixed-precision solves on this one  */
} cola_solve_info;

/* Solve A X = B for nrhs right-hand sides (packed, float64, device).
 *  - prec == COLA_PREC_FP64: textbook CG in FP64 to tol on the recursive
 *    residual, from x0 = 0 or the caller's X (x0_given); one FP64 product of
 *    the returned X gives relres_true.
 *  - prec == the op's working precision: mixed precision with an FP64
 *    residual formed from the FP64 factors, stopping when the FP64 relative
 *    residual <= tol.  refine == COLA_REFINE_RELIABLE (default): a single CG in
 *    the working precision whose x is folded into the FP64 solution and whose
 *    residual is replaced by the FP64 one every time it has dropped by
 *    inner_tol (or has converged), keeping the search direction; the
 *    replacement comes at the end of the check_every chunk in which the drop
 *    happened, and a right-hand side whose recursive residual falls below
 *    1e-5 of its last FP64 one stops iterating until then (its FP32
 *    recursion is rounding noise that far down).
 *    refine == COLA_REFINE_RESTART: each sweep solves A d = r / ||r|| from
 *    scratch to inner_tol and updates x += ||r|| d in FP64.
 * Right-hand sides converge independently; the call ends when all have
 * converged or hit a limit (the multi-RHS semantics of the paper's block
 * solves, App. D.5).  info: device array of nsys*nrhs entries, or NULL.
 * A warm start or a residual history takes the general multi-kernel path for
 * ops of many small systems (the resident batched kernel starts from zero and
 * records no history) and the separate-kernel path for the persistent fused CG
 * when a history is asked for.
 * The first call for a given nrhs allocates workspace (not capture-safe);
 * later calls with nrhs no larger allocate nothing. */
int32_t cola_cg_solve(cola_op_t op, const double* B, double* X, int32_t nrhs,
                      const cola_solve_opts* opts, cola_solve_info* info, void* stream);

/* Adjoint backward of X = A^{-1} B (App. B.2, rule 1).  Given X (the forward
 * solution) and G = dL/dX (packed float64), computes
 *     Lambda = A^{-1} G                     (= dL/dB), by a second solve,
 *     dK_jk  = - sum_r Lambda_r,(k) Z_r,(k)^T  with Z_r = X_r multiplied along
 *              every mode except k by term j's factors (mode-k unfoldings),
 *     dd     = - sum_r lambda_r * x_r   (elementwise),
 *     dsigma2= - sum_r lambda_r . x_r.
 * dfactors: HOST array with one device pointer per (system, term, factor), in
 * create order, each receiving an n_k x n_k float64 gradient (entry-wise,
 * unsymmetrised); NULL skips factor gradients.  ddiag: HOST array of nsys
 * device pointers (n_s float64 each; entries may be NULL), or NULL.
 * dsigma2: device array of nsys doubles, or NULL.  info as for the solve. */
int32_t cola_cg_solve_backward(cola_op_t op, const double* X, const double* G, int32_t nrhs,
                               const cola_solve_opts* opts, double* Lambda,
                               void* const* dfactors, void* const* ddiag, double* dsigma2,
                               cola_solve_info* info, void* stream);

/* Stochastic Lanczos quadrature estimate of log det A per system.  log det A
 * = Tr(Log(A)) for a symmetric positive definite A (App. A, derived
 * functions); stochastic Lanczos quadrature is the base-case iterative method
 * for such functions (App. C, table of base-case iterative algorithms).
 * Z: nprobes probe vectors per system (packed FP64 like B of cola_cg_solve,
 * device), e.g. Rademacher (+-1) entries, so that E[z z^T] = I.  One FP64 CG
 * over all probes (x0 = 0, at most max_iters iterations, stopping per probe
 * at ||r|| <= tol ||z||) records its step lengths and residual ratios; they
 * give each probe's Lanczos tridiagonal T (CG-Lanczos relation), and the
 * device forms est = ||z||^2 e1^T log(T) e1 by Gauss quadrature and
 * logdet = mean of est.
 *   X:      NULL, or device FP64 (packed like Z) receiving A^{-1} Z (the
 *           gradient of log det from the same probes is cola_logdet_grad,
 *           which can warm-start from this X);
 *   logdet: device array of nsys doubles;
 *   est:    NULL, or device array of nsys * nprobes per-probe estimates (NaN
 *           for a probe whose CG broke down);
 *   info:   NULL, or the per-probe CG outcome as for cola_cg_solve.
 * 1 <= max_iters <= 2048.  Enqueued on `stream`; the host waits on it every
 * 32 iterations to stop early.  The first call for a given nprobes and
 * max_iters allocates workspace. */
int32_t cola_slq_logdet(cola_op_t op, const double* Z, int32_t nprobes, double tol, int32_t max_iters,
                        double* X, double* logdet, double* est, cola_solve_info* info, void* stream);

/* Gradient of log det A per system (App. A: log det A = Tr(Log(A)); its derivative
 * Tr(A^{-1} dA/dtheta), estimated with probes as in Sec. 4's GP training): the
 * Hutchinson estimate (1/N) sum_z (A^{-1} z)^T (dA/dtheta) z over the N = nprobes
 * probe vectors Z (packed like B of cola_cg_solve, e.g. Rademacher), i.e. the solve
 * VJP of App. B.2 with X = G = Z, negated and divided by N inside the library.
 *   Lambda:   device FP64 like Z, receives A^{-1} Z (an ordinary cola_cg_solve with
 *             opts, which may warm-start from it, e.g. with the X of cola_slq_logdet);
 *   dfactors, ddiag, dsigma2, info: as for cola_cg_solve_backward.
 * Enqueued on `stream`; the first call for a given nprobes allocates workspace. */
int32_t cola_logdet_grad(cola_op_t op, const double* Z, int32_t nprobes, const cola_solve_opts* opts,
                         double* Lambda, void* const* dfactors, void* const* ddiag, double* dsigma2,
                         cola_solve_info* info, void* stream);

/* Diag(A) of every system, exactly: Diag(A + B) = Diag(A) + Diag(B) and
 * Diag(A (x) B) = vec(Diag(A) Diag(B)^T) (App. A, diagonal rules; row-major
 * vec), plus d and sigma2.  out: device FP64, n_total entries packed by system
 * (system i at its offset, as one right-hand side of cola_cg_solve).  O(n) per
 * term; enqueued on `stream`. */
int32_t cola_op_diagonal(cola_op_t op, double* out, void* stream);

/* probe estimators of Diag(A) (cola_diag_estimate.mode) */
#define COLA_DIAG_HUTCHINSON 0   /* (1/N) sum_j z_j . A z_j, every probe shared by all terms (Sec. 3.3) */
#define COLA_DIAG_DOUBLY     1   /* (1/N) sum_j sum_i z_ij . A_i z_ij over the Kronecker terms A_i, a
                                    probe set of its own per term, plus the exact d + sigma2 (App. B.1) */

/* Stochastic estimate of Diag(A) from MVMs with probe vectors (any entries
 * of identity covariance, e.g. +-1), all in FP64 on the device.
 *   Z:    device FP64 probes.  HUTCHINSON: packed like the right-hand sides of
 *         cola_cg_solve with nrhs = nprobes (system i: nprobes vectors of n_i).
 *         DOUBLY: system i holds nterms_i * nprobes vectors of n_i, term-major
 *         (term j's nprobes vectors together), systems in order.
 *   out:  device FP64, n_total entries packed by system (as cola_op_diagonal).
 * The sum's terms are applied one at a time through the same MVM kernels.
 * Enqueued on `stream`; the first call for a given nprobes allocates workspace. */
int32_t cola_diag_estimate(cola_op_t op, const double* Z, int32_t nprobes, int32_t mode, double* out,
                           void* stream);

/* Direct solve X = A^{-1} B of single-term systems A = K_1 (x) .. (x) K_F +
 * sigma2 * I by the Kronecker eigenvalue rules (App. A: the eigenvectors of a
 * Kronecker product are the Kronecker products of the factors' eigenvectors
 * and its eigenvalues the products of theirs; Sec. 3 dispatches solves of
 * such structure this way instead of iterating):
 *     X = (Q_1 (x) .. (x) Q_F) [ ((Q_1 (x) .. (x) Q_F)^T B) ./ (lam_1 (x) .. (x) lam_F + sigma2) ].
 * The factors must be symmetric positive semi-definite.  The first call
 * decomposes every factor on the device (FP64 one-sided Jacobi; it waits on
 * the stream once per sweep) and keeps the eigenvectors; later calls are two
 * FP64 Kronecker MVMs and one scaling, enqueued on `stream`.  B and X are
 * packed FP64 vectors as for cola_cg_solve and must not overlap.  Returns
 * COLA_ERR_UNSUPPORTED if any system has more than one term or a diagonal. */
int32_t cola_eig_solve(cola_op_t op, const double* B, double* X, int32_t nrhs, void* stream);

/* Pick kernel tile shapes for this op and nrhs by timing the candidates on
 * `stream` (synchronises it).  Optional: without it a fixed default is used. */
int32_t cola_autotune(cola_op_t op, int32_t nrhs, void* stream);

/* The op's tuned tile table as text, to keep a tuning cache across processes and ops of the same
 * shapes: a line "device <arch> <compute units>", then one line per tuned pass,
 * "<prec> <rows> <mode size> <inner extent> <leading extent> <wm> <wn>".  buf NULL: *len
 * receives the length (without the terminating NUL) and nothing is written; otherwise buf (cap
 * bytes) receives the NUL-terminated text, COLA_ERR_INVALID_ARG if it does not fit.  For callers
 * that cache tuning results. */
int32_t cola_autotune_export(cola_op_t op, char* buf, int64_t cap, int64_t* len);

/* Load a table written by cola_autotune_export (by this or another op): entries recorded on the
 * same device architecture and compute-unit count replace the op's own (synchronises the device
 * and drops captured chunk graphs); entries of another device are read and ignored.
 * COLA_ERR_INVALID_ARG for a malformed line or an invalid tile; nothing is applied then. */
int32_t cola_autotune_import(cola_op_t op, const char* text);

/* Engine switches.  Every engine is on by default and is used wherever its
 * shape conditions hold; switched off, the op uses the general per-mode
 * contraction path for those shapes instead (the same arithmetic up to
 * rounding order: for comparing engines and testing the general path).
 * Synchronises the device and drops captured chunk graphs.  Returns
 * COLA_ERR_INVALID_ARG for an unknown engine. */
#define COLA_ENGINE_FUSED_CG 1  /* persistent CG, one cooperative launch per chunk of iterations:
                                   one-term K1 (x) K2 (x) K3 (+ diag) with 64-wide modes, FP32
                                   working precision, no residual history.  With check_every
                                   = 0 every chunk of 128 iterations is enqueued up front
                                   (capture-safe); a barrier time-out, which a captured launch
                                   can meet if other work shares the GPU, is then reported
                                   as COLA_ERR_HIP in every right-hand side's info          */
#define COLA_ENGINE_GEMM2    2  /* dense-GEMM MVM: BF16, two-mode, modes multiples of 256       */
#define COLA_ENGINE_GEMM3    3  /* dense-GEMM MVM: FP32 or BF16x3, one-term three-mode, 256-wide
                                   modes                                                     */
#define COLA_ENGINE_SLAB     4  /* fused mode-2/mode-3 products of three-mode terms, modes <= 64 */
#define COLA_ENGINE_RESIDENT 5  /* resident batched CG of many small two-mode systems           */
#define COLA_ENGINE_SMALL64  6  /* FP64 solves of one-term two-mode systems with modes <= 64: the
                                   whole CG of each (system, RHS) in one workgroup (no precond) */
#define COLA_ENGINE_GEMM64   7  /* FP64 passes (residuals of mixed precision, FP64 CG, FP64
                                   products) of two-mode operators with modes multiples of 256
                                   as two dense FP64 GEMMs                                    */
int32_t cola_op_set_engine(cola_op_t op, int32_t engine, int32_t enable);

/* Per-kernel timing with HIP events recorded on the launch stream around
 * every kernel of the named class.  Classes: "slab23" (fused modes 2-3 of
 * three-mode terms), "contract_rows" (last mode), "contract_mid" (middle
 * mode), "contract_last" (first mode, with the diagonal term and the CG
 * epilogue), "update" (x, r update and residual norm), "resident" (batched
 * small systems), "cg_fused" (one launch of the persistent CG: a chunk of
 * iterations for a batch of right-hand sides), "gemm_pack", "gemm_mode3",
 * "gemm_mode2", "gemm_mode1" (the dense-GEMM engines' passes); the same names with "_fp64" for
 * launches in FP64 (plain FP64 solves and the FP64 residuals of mixed precision).  enable != 0
 * starts collecting (and clears totals). */
int32_t cola_profile_enable(cola_op_t op, int32_t enable);
/* Totals since enable: summed milliseconds and launch count for `kernel`;
 * synchronises the device.  Unknown names report zero launches. */
int32_t cola_profile_read(cola_op_t op, const char* kernel, double* total_ms, int64_t* launches);

/* Host-side ranges of every entry point (and of each system's solve, reliable update and
 * final fold) as roctx ranges, for rocprofv3 --marker-trace: on for enable != 0, process-wide,
 * off by default (a disabled range costs one atomic load).  For the callers that profile.
 * Always returns COLA_OK. */
int32_t cola_trace_enable(int32_t enable);

/* Static description of a status code. */
const char* cola_status_string(int32_t status);

#ifdef __cplusplus
}
#endif
#endif /* COLA_H */
