"""Pins for the oracle's direct solves, CG and refinement (CPU only)."""
from fractions import Fraction

import numpy as np
import pytest

import exact_ref as ex
import workloads as wl
from oracle import cg, direct, kron, lowprec


def _spd_terms(rng, dims, nterms=1):
    return [[wl.wishart_factor(rng, m) for m in dims] for _ in range(nterms)]


def test_cholesky_matches_exact_gaussian_elimination():
    K1 = [[4, 1], [1, 3]]
    K2 = [[2, 1, 0], [1, 3, 1], [0, 1, 2]]
    A = ex.add_diag(ex.kron(ex.frac_matrix(K1), ex.frac_matrix(K2)), [Fraction(1, 2)] * 6)
    b = [Fraction(v) for v in (1, -2, 3, 0, 5, -1)]
    x_exact = ex.solve(A, b)
    x = direct.cholesky_solve([[np.array(K1, float), np.array(K2, float)]],
                              np.array([[1, -2, 3, 0, 5, -1]], float), sigma2=0.5)
    assert np.allclose(x[0], [float(v) for v in x_exact], rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("dims", [(3, 4), (2, 3, 4), (5,)])
def test_kron_eigenvalues_are_products(dims):
    rng = np.random.default_rng(21)
    fs = [wl.wishart_factor(rng, m) for m in dims]
    lam_dense = np.sort(np.linalg.eigvalsh(kron.dense_kron(fs)))
    lam_rule = np.sort(direct.kron_eigenvalues(fs))
    assert np.allclose(lam_rule, lam_dense, rtol=1e-12, atol=1e-12 * lam_dense.max())


@pytest.mark.parametrize("dims", [(4, 5), (3, 4, 3)])
def test_kron_eig_solve_matches_cholesky(dims):
    rng = np.random.default_rng(22)
    terms = _spd_terms(rng, dims)
    B = rng.standard_normal((3, int(np.prod(dims))))
    x1 = direct.cholesky_solve(terms, B, 0.05)
    x2 = direct.kron_eig_solve(terms[0], B, 0.05)
    assert np.allclose(x1, x2, rtol=1e-11, atol=1e-11 * np.abs(x1).max())


def test_condition_number_matches_dense():
    rng = np.random.default_rng(23)
    terms = [[wl.rbf_kernel(np.sort(rng.uniform(0, 1, 6)), 0.3), wl.rbf_kernel(np.sort(rng.uniform(0, 1, 5)), 0.3)]]
    ev = np.linalg.eigvalsh(kron.dense_operator(terms, 0.1))
    assert np.isclose(direct.condition_number(terms[0], 0.1), ev.max() / ev.min(), rtol=1e-8)


def test_cg_matches_exact_arithmetic_cg_and_terminates():
    # Exact CG on an SPD 6x6 Kronecker system reaches the exact solution in <= 6 steps;
    # the float64 oracle must follow the same iterates (a sign or index slip would not).
    K1 = [[3, 1], [1, 2]]
    K2 = [[4, 1, 1], [1, 3, 0], [1, 0, 2]]
    A = ex.add_diag(ex.kron(ex.frac_matrix(K1), ex.frac_matrix(K2)), [Fraction(1)] * 6)
    b = [Fraction(v) for v in (1, 2, -1, 0, 3, 1)]
    xs = ex.cg(A, b, 6)
    assert xs[-1] == ex.solve(A, b)
    terms = [[np.array(K1, float), np.array(K2, float)]]
    res = cg.cg(lambda V: kron.mvm(terms, V, 1.0), np.array([[1, 2, -1, 0, 3, 1]], float),
                tol=0.0, max_iters=len(xs) - 1, keep_history=True)
    for k, xk in enumerate(xs):
        assert np.allclose(res.history["X"][k][0], [float(v) for v in xk], rtol=1e-11, atol=1e-12)


def test_cg_scaled_identity_one_iteration():
    B = np.random.default_rng(24).standard_normal((2, 12))
    res = cg.cg(lambda V: 2.5 * V, B, tol=1e-14, max_iters=10)
    assert list(res.iters) == [1, 1]
    assert np.allclose(res.X, B / 2.5, rtol=1e-15, atol=1e-15)


def test_cg_k_distinct_eigenvalues_k_iterations():
    # A diagonal operator with 3 distinct eigenvalues: CG's Krylov space holds the
    # exact solution after 3 steps.
    dvals = np.repeat([1.0, 4.0, 9.0], 5)
    B = np.random.default_rng(25).standard_normal((1, 15))
    res = cg.cg(lambda V: V * dvals[None, :], B, tol=1e-12, max_iters=50)
    assert res.iters[0] == 3
    assert np.allclose(res.X[0], B[0] / dvals, rtol=1e-12)


def test_cg_invariants_on_rbf_kron():
    rng = np.random.default_rng(26)
    terms = [[wl.rbf_kernel(np.sort(rng.uniform(0, 1, 6)), 0.3), wl.rbf_kernel(np.sort(rng.uniform(0, 1, 6)), 0.3)]]
    A = kron.dense_operator(terms, 0.1)
    b = rng.standard_normal((1, 36))
    xstar = np.linalg.solve(A, b[0])
    res = cg.cg(lambda V: kron.mvm(terms, V, 0.1), b, tol=0.0, max_iters=8, keep_history=True)
    R, P, X = res.history["R"], res.history["P"], res.history["X"]
    for i in range(6):
        for j in range(i + 1, 6):
            assert abs(R[i][0] @ R[j][0]) <= 1e-8 * np.linalg.norm(R[i][0]) * np.linalg.norm(R[j][0])
            assert abs(P[i][0] @ A @ P[j][0]) <= 1e-8 * np.sqrt((P[i][0] @ A @ P[i][0]) * (P[j][0] @ A @ P[j][0]))
    errs = [np.sqrt((X[k][0] - xstar) @ A @ (X[k][0] - xstar)) for k in range(len(X))]
    assert all(errs[k + 1] < errs[k] for k in range(len(errs) - 1))


def test_cg_converges_to_cholesky_on_c1_recipe_small():
    w = wl.config1(m=12)
    s = w.systems[0]
    res = cg.cg(lambda V: kron.mvm(s.factors, V, s.sigma2), w.B[0], tol=1e-12, max_iters=500)
    assert res.status == ["ok"]
    x = direct.cholesky_solve(s.factors, w.B[0], s.sigma2)
    assert np.allclose(res.X, x, rtol=1e-8, atol=1e-8 * np.abs(x).max())
    assert kron.relres(s.factors, res.X, w.B[0], s.sigma2)[0] <= 1e-12


def test_cg_status_edge_cases():
    n = 8
    B = np.zeros((4, n))
    B[1, 0] = np.nan
    B[2] = 1.0
    B[3] = np.arange(n) + 1.0
    # indefinite operator: diag with a negative entry
    dvals = np.ones(n)
    dvals[3] = -1.0
    res = cg.cg(lambda V: V * dvals[None, :], B, tol=1e-10, max_iters=20)
    assert res.status[0] == "ok" and res.iters[0] == 0 and not res.X[0].any()
    assert res.status[1] == "nonfinite"
    # p0 = 1: p0.Ap0 = 6 > 0; by hand p1 = (4/9 x7, 28/9) and p1.Ap1 = (112 - 784)/81 < 0
    assert res.status[2] == "not_spd" and res.iters[2] == 1
    # max_iters = 1 leaves a valid partial iterate
    res1 = cg.cg(lambda V: V * np.linspace(1, 10, n)[None, :], B[3:], tol=1e-12, max_iters=1)
    assert res1.status == ["not_converged"] and res1.iters[0] == 1
    assert np.all(np.isfinite(res1.X))


def test_refinement_fp32_inner_reaches_fp64_accuracy():
    rng = np.random.default_rng(27)
    terms = [[wl.rbf_kernel(np.sort(rng.uniform(0, 1, 10)), 0.2), wl.rbf_kernel(np.sort(rng.uniform(0, 1, 10)), 0.2)]]
    B = rng.standard_normal((2, 100))
    low = [[lowprec.to_fp32(f) for f in terms[0]]]
    res = cg.refine(lambda V: kron.mvm(terms, V, 0.01), lambda V: kron.mvm(low, V, 0.01), B,
                    tol=1e-12, inner_tol=1e-4, max_sweeps=20, inner_max_iters=2000)
    assert res.status == ["ok", "ok"]
    assert np.all(kron.relres(terms, res.X, B, 0.01) <= 1e-12)
    x = direct.cholesky_solve(terms, B, 0.01)
    assert np.allclose(res.X, x, rtol=1e-8, atol=1e-8 * np.abs(x).max())


def test_refinement_stagnates_with_wrong_inner_operator():
    B = np.ones((1, 6))
    # the inner operator is 2.25 A: each sweep leaves r_new = (1 - 1/2.25) r = 0.56 r,
    # which fails to halve the residual twice in a row
    res = cg.refine(lambda V: 2.0 * V, lambda V: 2.25 * 2.0 * V, B, tol=1e-10, inner_tol=1e-12,
                    max_sweeps=10, inner_max_iters=10)
    assert res.status == ["stagnated"]
