"""Pins of the preconditioned-CG and diagonal-estimator oracle against facts fixed by the mathematics:

* PCG with M = I takes the iterates of plain CG (the textbook CG oracle, an independent routine);
* PCG with Jacobi M = D takes the iterates of plain CG on the symmetrically scaled system
  D^{-1/2} A D^{-1/2} y = D^{-1/2} b mapped back by x = D^{-1/2} y (the PCG / split-preconditioning
  equivalence), step by step;
* PCG with M = A ends after one step with the exact solution; the Kronecker-eigen preconditioner of a
  one-term operator plus sigma2 I is that case; its trace-matching shift equals Tr(A - term 1) / n of
  the dense matrices;
* converged PCG solutions equal the dense Cholesky solution;
* the probe estimators of the diagonal are exact where the mathematics says so (Rademacher probes on a
  diagonal matrix), their means fall within the closed-form standard error of the exact diagonal, and
  the empirical per-entry variances over many probes match the closed forms, for Hutchinson on the sum
  and for the doubly stochastic estimator (sum of the terms' variances).
"""
import numpy as np

import workloads as wl
from oracle import cg, direct, kron, precond


def _sys(rng, dims, nterms, diag, sigma2):
    return wl.random_system(rng, dims, nterms=nterms, diag=diag, sigma2=sigma2)


def _A(s):
    return lambda V: kron.mvm(s.factors, V, s.sigma2, s.diag)


def test_pcg_identity_is_cg():
    rng = np.random.default_rng(81)
    s = _sys(rng, (6, 5, 4), 2, True, 0.1)
    B = rng.standard_normal((2, s.n))
    for k in (1, 3, 9):
        Xp, itp, _ = precond.pcg(_A(s), lambda R: R.copy(), B, 0.0, k)
        res = cg.cg(_A(s), B, 0.0, max_iters=k)
        assert list(itp) == [k, k]
        np.testing.assert_allclose(Xp, res.X, rtol=0, atol=1e-12 * np.abs(res.X).max())


def test_jacobi_pcg_is_cg_on_scaled_system():
    rng = np.random.default_rng(82)
    s = _sys(rng, (7, 6), 2, True, 0.05)
    s.diag[:] = rng.uniform(0.1, 20.0, size=s.n)            # a diagonal that dominates unevenly
    A = kron.dense_operator(s.factors, s.sigma2, s.diag)
    dinv = precond.jacobi_inverse(s.factors, s.sigma2, s.diag)
    np.testing.assert_allclose(1.0 / dinv, np.diag(A), rtol=1e-14)
    sc = np.sqrt(dinv)
    As = sc[:, None] * A * sc[None, :]
    b = rng.standard_normal((1, s.n))
    for k in (1, 2, 5, 12):
        Xp, _, _ = precond.pcg(_A(s), lambda R: R * dinv, b, 0.0, k)
        Y = cg.cg(lambda V: V @ As.T, b * sc, 0.0, max_iters=k).X
        np.testing.assert_allclose(Xp, Y * sc, rtol=0, atol=1e-10 * np.abs(Xp).max())


def test_pcg_exact_preconditioner_one_step_and_kron_eig_case():
    rng = np.random.default_rng(83)
    s = _sys(rng, (5, 4, 3), 1, False, 0.2)
    A = kron.dense_operator(s.factors, s.sigma2)
    B = rng.standard_normal((2, s.n))
    Xd = np.linalg.solve(A, B.T).T
    X, it, st = precond.pcg(_A(s), lambda R: np.linalg.solve(A, R.T).T, B, 1e-12, 50)
    assert list(it) == [1, 1] and st == ["ok", "ok"]
    np.testing.assert_allclose(X, Xd, rtol=0, atol=1e-11 * np.abs(Xd).max())
    assert precond.kron_eig_shift(s.factors, s.sigma2) == s.sigma2
    X, it, st = precond.pcg(_A(s), precond.kron_eig_preconditioner(s.factors, s.sigma2), B, 1e-12, 50)
    assert list(it) == [1, 1] and st == ["ok", "ok"]
    np.testing.assert_allclose(X, Xd, rtol=0, atol=1e-11 * np.abs(Xd).max())


def test_kron_eig_shift_is_trace_of_remainder_and_pcg_matches_cholesky():
    rng = np.random.default_rng(84)
    s = _sys(rng, (6, 5), 3, True, 0.3)
    A = kron.dense_operator(s.factors, s.sigma2, s.diag)
    first = kron.dense_kron(s.factors[0])
    c = precond.kron_eig_shift(s.factors, s.sigma2, s.diag)
    assert abs(c - np.trace(A - first) / s.n) <= 1e-13 * abs(c)
    B = rng.standard_normal((3, s.n))
    Xd = direct.cholesky_solve(s.factors, B, s.sigma2, s.diag)
    for Minv in (precond.kron_eig_preconditioner(s.factors, s.sigma2, s.diag),
                 lambda R: R * precond.jacobi_inverse(s.factors, s.sigma2, s.diag)):
        X, it, st = precond.pcg(_A(s), Minv, B, 1e-12, 500)
        assert st == ["ok"] * 3
        assert np.all(kron.relres(s.factors, X, B, s.sigma2, s.diag) <= 1e-12)
        np.testing.assert_allclose(X, Xd, rtol=0, atol=1e-9 * np.abs(Xd).max())


def test_diagonal_estimators_exact_cases_means_and_variances():
    rng = np.random.default_rng(85)
    # Rademacher probes on a diagonal operator: every probe gives the exact diagonal
    d = rng.uniform(0.1, 1.0, size=30)
    Z = wl.rademacher_probes(rng, 3, 30)
    np.testing.assert_allclose(precond.hutchinson_diagonal(lambda V: V * d, Z), d, rtol=1e-15)
    # a three-term Kronecker sum: closed-form variances against many probes
    s = _sys(rng, (4, 3), 3, False, 0.0)
    terms = [kron.dense_kron(fs) for fs in s.factors]
    A = sum(terms)
    exact = kron.operator_diagonal(s.factors)
    N = 20000
    Z = wl.rademacher_probes(rng, N, s.n)
    per_h = Z * (Z @ A.T)                                    # one row per probe
    Zs = [wl.rademacher_probes(rng, N, s.n) for _ in terms]
    per_d = sum(Zi * (Zi @ T.T) for Zi, T in zip(Zs, terms))
    var_h = precond.probe_variance(A)
    var_d = sum(precond.probe_variance(T) for T in terms)
    for per, var in ((per_h, var_h), (per_d, var_d)):
        mean = per.mean(axis=0)
        assert np.all(np.abs(mean - exact) <= 4.5 * np.sqrt(var / N) + 1e-12)
        emp = per.var(axis=0, ddof=1)
        # sample variance of N draws: relative standard error about sqrt(2 / N) for light tails
        assert np.all(np.abs(emp - var) <= 0.1 * var + 1e-12)
    # the library-style estimators agree with the per-probe means
    np.testing.assert_allclose(precond.hutchinson_diagonal(lambda V: V @ A.T, Z), per_h.mean(axis=0), rtol=1e-12)
    np.testing.assert_allclose(precond.doubly_stochastic_diagonal([lambda V, T=T: V @ T.T for T in terms], Zs),
                               per_d.mean(axis=0), rtol=1e-12)
    # Gaussian probes: the closed form A_kk^2 + sum_l A_kl^2
    G = rng.standard_normal((N, s.n))
    emp = (G * (G @ A.T)).var(axis=0, ddof=1)
    vg = precond.probe_variance(A, "gaussian")
    assert np.all(np.abs(emp - vg) <= 0.15 * vg)
