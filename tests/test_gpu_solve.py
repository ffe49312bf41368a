"""GPU parity of cola_cg_solve (plain FP64 CG and mixed-precision refinement) against the oracle."""
import numpy as np
import pytest

import workloads as wl
from oracle import cg as ocg
from oracle import direct, kron

pytestmark = pytest.mark.gpu


def _solve(systems, Bs, prec, nrhs, **kw):
    from gpu_util import infos, make_op, pack, unpack
    op = make_op(systems, prec="fp32" if prec == "fp64" else prec)
    X, info = op.solve(pack(Bs), nrhs, prec=prec, **kw)
    out = unpack(X, systems, nrhs), infos(info, len(systems) * nrhs)
    op.close()
    return out


def test_fp64_cg_c1_recipe_reduced():
    w = wl.config1(m=24)
    s = w.systems[0]
    (X,), info = _solve(w.systems, w.B, "fp64", 1, tol=1e-10, max_iters=3000)
    assert info[0]["status"] == 0
    assert kron.relres(s.factors, X, w.B[0], s.sigma2)[0] <= 1e-10
    xref = direct.cholesky_solve(s.factors, w.B[0], s.sigma2)
    kappa = direct.condition_number(s.factors[0], s.sigma2)
    assert np.linalg.norm(X - xref) <= 2 * kappa * 1e-10 * np.linalg.norm(xref)
    # same recurrence as the oracle: iteration counts agree closely
    ref = ocg.cg(lambda V: kron.mvm(s.factors, V, s.sigma2), w.B[0], 1e-10, 3000)
    assert abs(info[0]["iters"] - int(ref.iters[0])) <= max(3, int(0.05 * ref.iters[0]))


def test_fp64_cg_c1_full_size():
    w = wl.config1()
    s = w.systems[0]
    (X,), info = _solve(w.systems, w.B, "fp64", 1, tol=1e-10, max_iters=2000)
    assert info[0]["status"] == 0
    assert kron.relres(s.factors, X, w.B[0], s.sigma2)[0] <= 1e-10
    xref = direct.cholesky_solve(s.factors, w.B[0], s.sigma2)
    assert np.linalg.norm(X - xref) <= 1e-6 * np.linalg.norm(xref)


@pytest.mark.parametrize("prec,refine,inner", [("fp32", "reliable", 0.1), ("bf16x3", "reliable", 0.1),
                                               ("fp32", "restart", 1e-4), ("bf16x3", "restart", 1e-4)])
def test_refined_c2_recipe_reduced(prec, refine, inner):
    w = wl.config2(m=16, nrhs=4)
    s = w.systems[0]
    (X,), info = _solve(w.systems, w.B, prec, 4, tol=1e-6, max_iters=5000, inner_tol=inner, max_sweeps=40,
                        refine=refine)
    assert all(i["status"] == 0 for i in info), info
    rr = kron.relres(s.factors, X, w.B[0], s.sigma2)
    assert np.all(rr <= 1e-6), rr
    xref = direct.kron_eig_solve(s.factors[0], w.B[0], s.sigma2)
    kappa = direct.condition_number(s.factors[0], s.sigma2)
    assert np.linalg.norm(X - xref) <= 2 * kappa * 1e-6 * np.linalg.norm(xref)
    for i, r in zip(info, rr):
        assert abs(i["relres"] - r) <= 1e-3 * r + 1e-15     # the library's own FP64 residual


def test_refined_sum_of_kron_with_diag_bf16():
    w = wl.config5(m=32, nterms=4, nrhs=3)
    s = w.systems[0]
    (X,), info = _solve(w.systems, w.B, "bf16", 3, tol=1e-6, max_iters=500, inner_tol=0.1)
    assert all(i["status"] == 0 for i in info), info
    assert np.all(kron.relres(s.factors, X, w.B[0], s.sigma2, s.diag) <= 1e-6)
    xref = direct.cholesky_solve(s.factors, w.B[0], s.sigma2, s.diag)
    assert np.linalg.norm(X - xref) <= 1e-4 * np.linalg.norm(xref)


def test_refined_bf16_dense_gemm_path():
    """Sum of two 256^2 Wishart Kronecker terms + diagonal: BF16 CG on the dense-GEMM MVM with FP64
    reliable updates reaches 1e-6 true residual, certified by the oracle."""
    w = wl.config5(m=256, nterms=2, nrhs=3)
    s = w.systems[0]
    (X,), info = _solve(w.systems, w.B, "bf16", 3, tol=1e-6, max_iters=500, inner_tol=0.1)
    assert all(i["status"] == 0 for i in info), info
    rr = kron.relres(s.factors, X, w.B[0], s.sigma2, s.diag)
    assert np.all(rr <= 1e-6), rr
    for i, r in zip(info, rr):
        assert abs(i["relres"] - r) <= 1e-3 * r + 1e-15


def test_refined_fp32_dense_gemm3_path():
    """256^3 Wishart-factor operator (condition number ~1e2, a few hundred iterations): FP32 CG on the
    three-GEMM MVM with FP64 reliable updates reaches 1e-6 true residual, certified by the oracle."""
    rng = np.random.default_rng(93)
    s = wl.random_system(rng, (256, 256, 256), nterms=1, diag=False, sigma2=0.5)
    B = rng.standard_normal((2, s.n))
    (X,), info = _solve([s], [B], "fp32", 2, tol=1e-6, max_iters=3000, inner_tol=0.1)
    assert all(i["status"] == 0 for i in info), info
    rr = kron.relres(s.factors, X, B, s.sigma2)
    assert np.all(rr <= 1e-6), rr
    for i, r in zip(info, rr):
        assert abs(i["relres"] - r) <= 1e-3 * r + 1e-15


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("iters", [1, 6, 40])
def test_gemm3_deferred_iterate_at_iteration_limit(iters, prec):
    """The three-GEMM engines apply x += alpha p one iteration late: the FP32 engine in its first
    pass, the BF16x3 engine (the direction alternating between two buffers) half in its middle and
    half in its last pass.  A solve stopped by the iteration limit must still contain its last step,
    also after reliable updates (the fold catches a pending step up from the right buffer, the update
    clears the flag, the next iteration resumes the deferral): the same solve on the contraction
    passes (x updated at once) agrees to FP32 rounding, while a dropped or doubled step, or a step
    taken from the wrong buffer, would differ by O(1); both are certified by the oracle's FP64
    residual of the returned X."""
    from gpu_util import infos, make_op, pack, unpack
    rng = np.random.default_rng(97)
    s = wl.random_system(rng, (256, 256, 256), nterms=1, diag=False, sigma2=0.5)
    B = rng.standard_normal((2, s.n))
    out = []
    for gemm3 in (True, False):
        op = make_op([s], prec=prec)
        op.set_engine("gemm3", gemm3)
        X, info = op.solve(pack([B]), 2, tol=1e-12, max_iters=iters, prec=prec, inner_tol=0.1)
        out.append((unpack(X, [s], 2)[0], infos(info, 2)))
        op.close()
    (Xg, ig), (Xc, ic) = out
    for i in ig + ic:
        assert i["status"] == 1 and i["iters"] == iters, i
        if iters >= 40:
            assert i["sweeps"] >= 1, i                      # a reliable update was crossed (they fall at chunk ends)
    assert np.abs(Xg - Xc).max() <= 1e-4 * np.abs(Xc).max()
    rr = kron.relres(s.factors, Xg, B, s.sigma2)
    for i, r in zip(ig, rr):
        assert abs(i["relres"] - r) <= 1e-3 * r + 1e-15


@pytest.mark.parametrize("tol", [1e-5, 1e-9])
def test_gemm3_direction_buffers_per_rhs(tol):
    """The BF16x3 engine keeps each right-hand side's direction in one of two buffers, flipped every
    iteration it takes.  A right-hand side that is an eigenvector of the operator (b = u1 (x) u2 (x) u3)
    has its recursive residual at rounding level after one step and pauses there (tol 1e-5: certified
    at once; tol 1e-9: the FP64 residual resumes it), while the random ones keep iterating, so their
    buffers part in parity.  Every right-hand side must come out as from the contraction passes (x
    updated at once): the same iteration counts up to the drift of a different summation order, the
    solutions equal to the tolerance's forward error, all certified by the oracle's FP64 residual."""
    from gpu_util import infos, make_op, pack, unpack
    rng = np.random.default_rng(99)
    s = wl.random_system(rng, (256, 256, 256), nterms=1, diag=False, sigma2=0.5)
    u = [np.linalg.eigh(f)[1][:, -1 - k] for k, f in enumerate(s.factors[0])]
    B = rng.standard_normal((3, s.n))
    B[1] = np.einsum("a,b,c->abc", *u).reshape(-1) * 3.0
    out = []
    for gemm3 in (True, False):
        op = make_op([s], prec="bf16x3")
        op.set_engine("gemm3", gemm3)
        X, info = op.solve(pack([B]), 3, tol=tol, max_iters=2000, prec="bf16x3", inner_tol=0.1, check_every=4)
        out.append((unpack(X, [s], 3)[0], infos(info, 3)))
        op.close()
    (Xg, ig), (Xc, ic) = out
    rr = kron.relres(s.factors, Xg, B, s.sigma2)
    for k in range(3):
        assert ig[k]["status"] == 0 and ic[k]["status"] == 0, (ig, ic)
        assert abs(ig[k]["iters"] - ic[k]["iters"]) <= max(2, ic[k]["iters"] // 20), (ig, ic)
        assert rr[k] <= tol and abs(ig[k]["relres"] - rr[k]) <= 1e-3 * rr[k], (rr, ig)
    assert ig[1]["iters"] < ig[0]["iters"] and ig[1]["iters"] < ig[2]["iters"], ig
    ev = [np.linalg.eigvalsh(f) for f in s.factors[0]]
    kappa = (np.prod([e.max() for e in ev]) + s.sigma2) / (np.prod([e.min() for e in ev]) + s.sigma2)
    for k in range(3):
        assert np.linalg.norm(Xg[k] - Xc[k]) <= 4 * kappa * tol * np.linalg.norm(Xc[k]), k


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_gemm3_cg_with_diagonal(prec):
    """The three-GEMM engines' CG epilogue with a diagonal d (q = K p + (sigma2 + d) p, then p.q),
    with the BF16x3 engine's alternating direction: a solve to 1e-9 certified by the oracle's FP64
    residual, within the forward-error bound of the contraction passes' solution, iteration counts
    within the drift of a different summation order; and the same solve stopped at 7 iterations
    agreeing with the contraction passes to FP32 rounding."""
    from gpu_util import infos, make_op, pack, unpack
    rng = np.random.default_rng(101)
    s = wl.random_system(rng, (256, 256, 256), nterms=1, diag=True, sigma2=0.3)
    B = rng.standard_normal((2, s.n))
    res = {}
    for gemm3 in (True, False):
        for tol, mi in ((1e-9, 3000), (1e-12, 7)):
            op = make_op([s], prec=prec)
            op.set_engine("gemm3", gemm3)
            X, info = op.solve(pack([B]), 2, tol=tol, max_iters=mi, prec=prec, inner_tol=0.1)
            res[(gemm3, mi)] = (unpack(X, [s], 2)[0], infos(info, 2))
            op.close()
    (Xg, ig), (Xc, ic) = res[(True, 3000)], res[(False, 3000)]
    rr = kron.relres(s.factors, Xg, B, s.sigma2, s.diag)
    ev = [np.linalg.eigvalsh(f) for f in s.factors[0]]
    lo = np.prod([e.min() for e in ev]) + s.sigma2 + s.diag.min()
    hi = np.prod([e.max() for e in ev]) + s.sigma2 + s.diag.max()
    for k in range(2):
        assert ig[k]["status"] == 0 and ic[k]["status"] == 0, (ig, ic)
        assert rr[k] <= 1e-9 and abs(ig[k]["relres"] - rr[k]) <= 1e-3 * rr[k], (rr, ig)
        assert abs(ig[k]["iters"] - ic[k]["iters"]) <= max(2, ic[k]["iters"] // 20), (ig, ic)
        assert np.linalg.norm(Xg[k] - Xc[k]) <= 4 * (hi / lo) * 1e-9 * np.linalg.norm(Xc[k])
    (Xg, ig), (Xc, ic) = res[(True, 7)], res[(False, 7)]
    for i in ig + ic:
        assert i["status"] == 1 and i["iters"] == 7, i
    assert np.abs(Xg - Xc).max() <= 1e-4 * np.abs(Xc).max()


@pytest.mark.parametrize("iters", [1, 5])
def test_gemm2_deferred_iterate_at_iteration_limit(iters):
    """The BF16 two-GEMM engine stopped at the iteration limit agrees with the BF16 contraction passes
    to BF16 rounding (a dropped or doubled step would differ by O(1)), and its reported residual is
    the oracle's FP64 residual of the returned X."""
    from gpu_util import infos, make_op, pack, unpack
    rng = np.random.default_rng(98)
    s = wl.random_system(rng, (256, 512), nterms=2, diag=True, sigma2=0.3)
    B = rng.standard_normal((3, s.n))
    out = []
    for gemm2 in (True, False):
        op = make_op([s], prec="bf16")
        op.set_engine("gemm2", gemm2)
        X, info = op.solve(pack([B]), 3, tol=1e-12, max_iters=iters, prec="bf16", inner_tol=0.1)
        out.append((unpack(X, [s], 3)[0], infos(info, 3)))
        op.close()
    (Xg, ig), (Xc, ic) = out
    for i in ig + ic:
        assert i["status"] == 1 and i["iters"] == iters, i
    assert np.abs(Xg - Xc).max() <= 2e-2 * np.abs(Xc).max()
    rr = kron.relres(s.factors, Xg, B, s.sigma2, s.diag)
    for i, r in zip(ig, rr):
        assert abs(i["relres"] - r) <= 1e-3 * r + 1e-15


def test_refined_uneven_batch_fp32():
    w = wl.config3(nsys=6, dmin=5, dmax=40)
    (Xs), info = _solve(w.systems, w.B, "fp32", 1, tol=1e-8, max_iters=3000)
    for s, X, B, i in zip(w.systems, Xs, w.B, info):
        assert i["status"] == 0
        assert kron.relres(s.factors, X, B, s.sigma2)[0] <= 1e-8
        xref = direct.kron_eig_solve(s.factors[0], B, s.sigma2)
        assert np.linalg.norm(X - xref) <= 2 * direct.condition_number(s.factors[0], s.sigma2) * 1e-8 * \
            np.linalg.norm(xref)


def test_status_edge_cases_match_oracle():
    rng = np.random.default_rng(41)
    s = wl.random_system(rng, (4, 6), sigma2=0.2)
    n = s.n
    B = rng.standard_normal((4, n))
    B[0] = 0.0                       # zero right-hand side: x = 0, no iterations
    B[1, 5] = np.nan                 # non-finite input
    (X,), info = _solve([s], [B], "fp64", 4, tol=1e-12, max_iters=500)
    ref = ocg.cg(lambda V: kron.mvm(s.factors, V, s.sigma2), B, 1e-12, 500)
    assert info[0]["status"] == 0 and info[0]["iters"] == 0 and not X[0].any()
    assert ref.status[0] == "ok"
    assert info[1]["status"] == -3 and ref.status[1] == "nonfinite"
    assert info[2]["status"] == 0 and info[3]["status"] == 0
    # iteration limit: valid partial iterate, NOT_CONVERGED
    (X1,), info1 = _solve([s], [B[2:3]], "fp64", 1, tol=1e-14, max_iters=2)
    assert info1[0]["status"] == 1 and info1[0]["iters"] == 2 and np.all(np.isfinite(X1))
    r1 = ocg.cg(lambda V: kron.mvm(s.factors, V, s.sigma2), B[2:3], 1e-14, 2)
    assert np.allclose(X1, r1.X, rtol=1e-10, atol=1e-12)


def test_indefinite_operator_reports_not_spd():
    rng = np.random.default_rng(42)
    K1 = np.diag([1.0, 2.0, -3.0])
    K2 = wl.wishart_factor(rng, 4)
    s = wl.System(factors=[[K1, K2]], sigma2=0.0)
    B = rng.standard_normal((1, 12))
    (X,), info = _solve([s], [B], "fp64", 1, tol=1e-12, max_iters=100)
    ref = ocg.cg(lambda V: kron.mvm(s.factors, V, 0.0), B, 1e-12, 100)
    assert ref.status[0] == "not_spd"
    assert info[0]["status"] == -2


def test_solve_is_deterministic():
    w = wl.config2(m=12, nrhs=2)
    a, ia = _solve(w.systems, w.B, "fp32", 2, tol=1e-6, max_iters=3000)
    b, ib = _solve(w.systems, w.B, "fp32", 2, tol=1e-6, max_iters=3000)
    assert np.array_equal(a[0], b[0]) and ia == ib


def test_no_poll_mode_matches_polling_mode():
    w = wl.config1(m=16)
    a, ia = _solve(w.systems, w.B, "fp64", 1, tol=1e-10, max_iters=400, check_every=0)
    b, ib = _solve(w.systems, w.B, "fp64", 1, tol=1e-10, max_iters=400, check_every=7)
    assert np.array_equal(a[0], b[0]) and ia == ib


def test_reliable_updates_match_fp64_iteration_count():
    """Reliable updates keep the Krylov space: iterations stay close to plain FP64 CG."""
    w = wl.config2(m=20, nrhs=2)
    s = w.systems[0]
    (X,), info = _solve(w.systems, w.B, "fp32", 2, tol=1e-8, max_iters=6000)
    ref = ocg.cg(lambda V: kron.mvm(s.factors, V, s.sigma2), w.B[0], 1e-8, 6000)
    assert all(i["status"] == 0 for i in info), info
    assert np.all(kron.relres(s.factors, X, w.B[0], s.sigma2) <= 1e-8)
    for i, k in zip(info, ref.iters):
        # FP32 recurrences lose orthogonality sooner than FP64 ones, so some delay is inherent
        assert i["iters"] <= 1.5 * k + 20, (i, k)
        assert i["sweeps"] >= 1


def test_reliable_no_poll_mode_matches_polling_mode():
    w = wl.config2(m=12, nrhs=2)
    a, ia = _solve(w.systems, w.B, "fp32", 2, tol=1e-7, max_iters=640, check_every=0)
    b, ib = _solve(w.systems, w.B, "fp32", 2, tol=1e-7, max_iters=640, check_every=32)
    assert np.array_equal(a[0], b[0]) and ia == ib
