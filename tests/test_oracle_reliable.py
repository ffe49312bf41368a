"""Pins for the oracle's reliable-update CG (CPU only).

The paper prints no mixed-precision scheme; the oracle writes out the reading the library builds.
These tests tie that reading to what mathematics fixes: without rounding it is textbook CG (a
residual replacement changes nothing then), with float32 vectors it reaches float64 accuracy where
plain float32 CG cannot, it replaces the residual once per factor delta of reduction, and an
inconsistent low-precision operator makes it stagnate.  Right-hand sides that converge within a
chunk (an eigenvector of the operator: one exact CG step) must not run on past the working
precision's noise floor, whatever the chunk length.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import cg, direct, kron, lowprec


def _rbf_terms(rng, m=10, ell=0.2):
    return [[wl.rbf_kernel(np.sort(rng.uniform(0, 1, m)), ell), wl.rbf_kernel(np.sort(rng.uniform(0, 1, m)), ell)]]


@pytest.mark.parametrize("delta,every", [(0.1, 1), (0.5, 7), (0.01, 3)])
def test_without_rounding_it_is_textbook_cg(delta, every):
    rng = np.random.default_rng(41)
    s = wl.random_system(rng, (7, 6), nterms=2, diag=True, sigma2=0.2)
    B = rng.standard_normal((3, s.n))
    A = lambda V: kron.mvm(s.factors, V, s.sigma2, s.diag)
    ref = cg.cg(A, B, tol=1e-10, max_iters=500)
    res = cg.reliable(A, A, B, tol=1e-10, delta=delta, max_iters=500, check_every=every, low_dtype=None)
    assert res.status == ["ok"] * 3
    assert np.all(np.abs(res.iters - ref.iters) <= 1), (res.iters, ref.iters)
    assert np.allclose(res.X, ref.X, rtol=1e-8, atol=1e-10 * np.abs(ref.X).max())
    assert np.all(res.relres_true <= 1e-10)


def test_float32_vectors_reach_float64_accuracy():
    """Plain float32 CG stalls near its rounding floor; reliable updates reach 1e-11 and the
    Cholesky solution within the forward-error bound."""
    rng = np.random.default_rng(42)
    terms = _rbf_terms(rng)
    low = [[lowprec.to_fp32(f) for f in terms[0]]]
    B = rng.standard_normal((2, 100))
    A64 = lambda V: kron.mvm(terms, V, 0.01)
    Alo = lambda V: kron.mvm(low, V, 0.01)
    plain = cg.cg(Alo, B, tol=1e-11, max_iters=3000, dtype=np.float32)
    assert np.all(kron.relres(terms, plain.X, B, 0.01) > 1e-9)
    res = cg.reliable(A64, Alo, B, tol=1e-11, delta=0.1, max_iters=3000, check_every=8)
    assert res.status == ["ok", "ok"]
    rr = kron.relres(terms, res.X, B, 0.01)
    assert np.all(rr <= 1e-11)
    assert np.allclose(res.relres_true, rr, rtol=1e-6)
    x = direct.cholesky_solve(terms, B, 0.01)
    kappa = float(np.linalg.cond(kron.dense_operator(terms, 0.01)))
    assert np.all(np.linalg.norm(res.X - x, axis=1) <= 2 * kappa * 1e-11 * np.linalg.norm(x, axis=1))


def test_one_replacement_per_factor_delta():
    """Replacing right after each trigger (check_every = 1) without rounding: every replacement but
    the last follows a fall of the recursive residual below delta times the previous true residual,
    and the last certifies convergence, so there are between 1 and ceil(log tol / log delta) + 1 of
    them; with delta ** 2 below tol the first fall already ends the solve (two at most).  The
    residual just after each replacement is the true one (relres_true = relres_recursive at the
    end).  (The replaced trajectory drifts from textbook CG's by rounding amplified over the
    iterations, so the exact trigger points are not compared.)"""
    rng = np.random.default_rng(43)
    s = wl.random_system(rng, (8, 8), nterms=1, diag=False, sigma2=0.5)
    B = rng.standard_normal((2, s.n))
    A = lambda V: kron.mvm(s.factors, V, s.sigma2)
    for delta, tol in ((0.1, 1e-8), (0.01, 1e-8), (0.3, 1e-6), (1e-5, 1e-8)):
        res = cg.reliable(A, A, B, tol=tol, delta=delta, max_iters=1000, check_every=1, low_dtype=None)
        k = int(np.ceil(np.log(tol) / np.log(delta) - 1e-9))
        assert res.status == ["ok", "ok"]
        assert np.all((res.updates >= 1) & (res.updates <= k + 1)), (delta, res.updates, k)
        assert np.allclose(res.relres_true, res.relres_recursive, rtol=1e-6)
        assert np.all(kron.relres(s.factors, res.X, B, s.sigma2) <= tol)


def test_edge_cases_and_stagnation():
    rng = np.random.default_rng(44)
    s = wl.random_system(rng, (6, 5), nterms=1, diag=True, sigma2=0.3)
    A = lambda V: kron.mvm(s.factors, V, s.sigma2, s.diag)
    B = rng.standard_normal((3, s.n))
    B[1] = 0.0
    res = cg.reliable(A, A, B, tol=1e-10, delta=0.1, max_iters=3, check_every=2)
    assert res.status[1] == "ok" and res.iters[1] == 0 and np.all(res.X[1] == 0.0)
    for i in (0, 2):
        assert res.status[i] == "not_converged" and res.iters[i] == 3
        # relative to the norm of b as the working precision holds it (float32 here)
        assert abs(res.relres_true[i] - kron.relres(s.factors, res.X[i:i + 1], B[i:i + 1], s.sigma2, s.diag)[0]) \
            <= 1e-6 * res.relres_true[i]
    # restarting the direction at every replacement still converges, never in fewer iterations
    ref = cg.cg(A, B[[0]], tol=1e-10, max_iters=500)
    rst = cg.reliable(A, A, B[[0]], tol=1e-10, delta=0.1, max_iters=500, check_every=1, low_dtype=None,
                      restart_dir=True)
    assert rst.status == ["ok"] and rst.iters[0] >= ref.iters[0]
    # an inner operator 2.25 A: with the direction restarted at each replacement every cycle
    # converges its recursion in one step while the true residual only shrinks to 1 - 1/2.25 of
    # itself, so the third such cycle in a row ends the solve as stagnated; keeping the direction,
    # the solve never reports convergence either
    Bs = np.ones((1, 6))
    bad = cg.reliable(lambda V: 2.0 * V, lambda V: 4.5 * V, Bs, tol=1e-10, delta=0.1, max_iters=200,
                      check_every=1, low_dtype=None, restart_dir=True)
    assert bad.status == ["stagnated"] and bad.updates[0] == 3 and bad.iters[0] == 3
    assert abs(bad.relres_true[0] - (1.0 - 1.0 / 2.25) ** 3) <= 1e-12
    kept = cg.reliable(lambda V: 2.0 * V, lambda V: 4.5 * V, Bs, tol=1e-10, delta=0.1, max_iters=200,
                       check_every=1, low_dtype=None)
    assert kept.status[0] in ("stagnated", "not_converged") and kept.relres_true[0] > 1e-10


@pytest.mark.parametrize("every", [1, 4, 32])
def test_eigenvector_rhs_converges_at_any_chunk_length(every):
    """b = 3 u1 (x) u2 (x) u3 with u_k eigenvectors of the factors: exact CG ends after one step with
    x = b / lambda.  In float32 the recursive residual is then at rounding level, and steps taken on
    it are noise; the right-hand side waits for its update there, so for every chunk length the
    solve reaches 1e-9 within a few iterations and returns b / lambda (forward error within
    kappa tol).  A random right-hand side beside it is unaffected (the same iterations to one)."""
    rng = np.random.default_rng(99)
    s = wl.random_system(rng, (16, 16, 16), nterms=1, diag=False, sigma2=0.5)
    pairs = [np.linalg.eigh(f) for f in s.factors[0]]
    u = [v[:, -1 - k] for k, (_, v) in enumerate(pairs)]
    lam = float(np.prod([w[-1 - k] for k, (w, _) in enumerate(pairs)])) + s.sigma2
    B = rng.standard_normal((2, s.n))
    B[1] = 3.0 * np.einsum("a,b,c->abc", *u).reshape(-1)
    low = [[lowprec.to_fp32(f) for f in s.factors[0]]]
    A64 = lambda V: kron.mvm(s.factors, V, s.sigma2)
    Alo = lambda V: kron.mvm(low, V, float(np.float32(s.sigma2)))
    res = cg.reliable(A64, Alo, B, tol=1e-9, delta=0.1, max_iters=2000, check_every=every)
    ref = cg.reliable(A64, Alo, B, tol=1e-9, delta=0.1, max_iters=2000, check_every=1)
    assert res.status == ["ok", "ok"], (res.status, res.iters)
    assert res.iters[1] <= 12, res.iters
    assert abs(int(res.iters[0]) - int(ref.iters[0])) <= 1
    ev = [w for w, _ in pairs]
    kappa = (np.prod([e.max() for e in ev]) + s.sigma2) / (np.prod([e.min() for e in ev]) + s.sigma2)
    x = B[1] / lam
    assert np.linalg.norm(res.X[1] - x) <= kappa * 1e-9 * np.linalg.norm(x)


def test_fast_solves_with_long_chunks_track_textbook_cg():
    """A system solved in ~45 iterations with 32-iteration chunks: each chunk's recursion would run
    far past the noise floor; waiting there keeps the iteration count within a few of textbook CG
    (running on gave 231 / 542 / 381 iterations before the rule)."""
    rng = np.random.default_rng(7002)
    s = wl.random_system(rng, (12, 10), nterms=2, diag=True, sigma2=0.2)
    B = rng.standard_normal((3, s.n))
    low = [[lowprec.to_fp32(f) for f in row] for row in s.factors]
    A64 = lambda V: kron.mvm(s.factors, V, s.sigma2, s.diag)
    Alo = lambda V: kron.mvm(low, V, float(np.float32(s.sigma2)), lowprec.to_fp32(s.diag))
    ref = cg.cg(A64, B, tol=1e-10, max_iters=500)
    res = cg.reliable(A64, Alo, B, tol=1e-10, delta=0.1, max_iters=3000, check_every=32)
    assert res.status == ["ok"] * 3
    assert np.all(res.iters <= ref.iters + 4), (res.iters, ref.iters)
    assert np.all(kron.relres(s.factors, res.X, B, s.sigma2, s.diag) <= 1e-10)
