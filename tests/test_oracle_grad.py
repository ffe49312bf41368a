"""Pins for the oracle's solve gradients and rounding emulator (CPU only)."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import direct, grad, kron, lowprec


def _problem(rng, dims, nterms, with_diag, nrhs=2, sigma2=0.3):
    terms = [[wl.wishart_factor(rng, m) for m in dims] for _ in range(nterms)]
    n = int(np.prod(dims))
    d = rng.uniform(0.1, 1.0, n) if with_diag else None
    B = rng.standard_normal((nrhs, n))
    W = rng.standard_normal((nrhs, n))
    X = direct.cholesky_solve(terms, B, sigma2, d)
    Lam = direct.cholesky_solve(terms, W, sigma2, d)       # lambda = A^{-1} dL/dx, A symmetric
    return terms, d, B, W, X, Lam, sigma2


@pytest.mark.parametrize("dims,nterms,with_diag", [((3, 4), 1, False), ((2, 3, 2), 1, True),
                                                   ((3, 3), 2, True), ((2, 2, 3), 2, False)])
def test_closed_forms_match_dense_chain_rule(dims, nterms, with_diag):
    rng = np.random.default_rng(31)
    terms, d, B, W, X, Lam, s2 = _problem(rng, dims, nterms, with_diag)
    g1 = grad.grad_dense(terms, X, Lam, with_diag)
    g2 = grad.grad_kron(terms, X, Lam, with_diag)
    for a, b in zip(g1[0], g2[0]):
        for fa, fb in zip(a, b):
            assert np.allclose(fa, fb, rtol=1e-11, atol=1e-12)
    if with_diag:
        assert np.allclose(g1[1], g2[1], rtol=1e-12, atol=1e-13)
    assert np.isclose(g1[2], g2[2], rtol=1e-12)


def test_two_factor_closed_form_written_out():
    # dK1 = -Lam K2 X^T and dK2 = -Lam^T K1 X in the row-major convention (one RHS)
    rng = np.random.default_rng(32)
    terms, d, B, W, X, Lam, s2 = _problem(rng, (3, 5), 1, False, nrhs=1)
    K1, K2 = terms[0]
    Xm, Lm = X[0].reshape(3, 5), Lam[0].reshape(3, 5)
    g = grad.grad_kron(terms, X, Lam)
    assert np.allclose(g[0][0][0], -Lm @ K2 @ Xm.T, rtol=1e-13, atol=1e-14)
    assert np.allclose(g[0][0][1], -Lm.T @ K1 @ Xm, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("dims,nterms,with_diag", [((3, 4), 1, True), ((2, 2, 3), 2, True)])
def test_closed_forms_match_finite_differences(dims, nterms, with_diag):
    rng = np.random.default_rng(33)
    terms, d, B, W, X, Lam, s2 = _problem(rng, dims, nterms, with_diag)
    dfac, dd, ds2 = grad.grad_kron(terms, X, Lam, with_diag)
    F = len(dims)
    for j in range(nterms):
        for k in range(F):
            m = dims[k]
            for (a, i) in [(0, 0), (m - 1, 0), (0, m - 1), (m // 2, (m + 1) // 2 % m)]:
                fd = grad.grad_fd(terms, s2, d, B, W, ("factor", j, k, a, i))
                assert np.isclose(fd, dfac[j][k][a, i], rtol=1e-6, atol=1e-8)
    for p in (0, int(np.prod(dims)) - 1):
        assert np.isclose(grad.grad_fd(terms, s2, d, B, W, ("diag", p)), dd[p], rtol=1e-6, atol=1e-8)
    assert np.isclose(grad.grad_fd(terms, s2, d, B, W, ("sigma2",)), ds2, rtol=1e-6, atol=1e-8)


def test_symmetric_pair_perturbation_is_sum_of_entries():
    # perturbing K[a,i] and K[i,a] together moves L by G[a,i] + G[i,a]
    rng = np.random.default_rng(34)
    terms, d, B, W, X, Lam, s2 = _problem(rng, (3, 3), 1, False)
    G = grad.grad_kron(terms, X, Lam)[0][0][0]
    h = 1e-5

    def L(delta):
        t = [[f.copy() for f in terms[0]]]
        t[0][0][0, 2] += delta
        t[0][0][2, 0] += delta
        return grad.loss(direct.cholesky_solve(t, B, s2), W)
    fd = (L(h) - L(-h)) / (2 * h)
    assert np.isclose(fd, G[0, 2] + G[2, 0], rtol=1e-6)


def test_lengthscale_chain_rule_matches_fd():
    rng = np.random.default_rng(35)
    p1, p2 = np.sort(rng.uniform(0, 1, 4)), np.sort(rng.uniform(0, 1, 5))
    l1, l2, s2 = 0.3, 0.25, 0.05
    B = rng.standard_normal((1, 20))
    W = rng.standard_normal((1, 20))

    def solve(a, b):
        return direct.cholesky_solve([[wl.rbf_kernel(p1, a), wl.rbf_kernel(p2, b)]], B, s2)
    terms = [[wl.rbf_kernel(p1, l1), wl.rbf_kernel(p2, l2)]]
    X = solve(l1, l2)
    Lam = direct.cholesky_solve(terms, W, s2)
    dK = grad.grad_kron(terms, X, Lam)[0][0]
    g1 = grad.rbf_lengthscale_grad(dK[0], terms[0][0], p1, l1)
    h = 1e-6
    fd = (grad.loss(solve(l1 + h, l2), W) - grad.loss(solve(l1 - h, l2), W)) / (2 * h)
    assert np.isclose(g1, fd, rtol=1e-6)


def test_bf16_rounding_textbook_ties():
    one = 1.0
    assert lowprec.to_bf16(np.array([one]))[0] == 1.0
    assert lowprec.to_bf16(np.array([1 + 2.0 ** -8]))[0] == 1.0                   # tie -> even (mantissa 0)
    assert lowprec.to_bf16(np.array([1 + 2.0 ** -7 + 2.0 ** -8]))[0] == 1 + 2.0 ** -6  # tie -> even (mantissa 2)
    assert lowprec.to_bf16(np.array([1 + 2.0 ** -8 + 2.0 ** -20]))[0] == 1 + 2.0 ** -7


def test_bf16_rounding_matches_torch():
    v = np.random.default_rng(36).standard_normal(10000) * 10.0 ** np.random.default_rng(37).uniform(-5, 5, 10000)
    ref = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(lowprec.to_bf16(v), ref)


def test_bf16_three_way_split_reaches_fp32_accuracy():
    v = np.random.default_rng(38).standard_normal(5000)
    f32 = lowprec.to_fp32(v)
    err = np.abs(lowprec.bf16_split_value(v, 3) - f32) / np.abs(f32)
    assert err.max() <= 2.0 ** -23
    err1 = np.abs(lowprec.bf16_split_value(v, 1) - f32) / np.abs(f32)
    assert err1.max() > 2.0 ** -10


def test_min_eig_rounded_matches_dense():
    rng = np.random.default_rng(39)
    fs = [wl.rbf_kernel(np.sort(rng.uniform(0, 1, 6)), 0.15) for _ in range(2)]
    lam = np.linalg.eigvals(kron.dense_kron([lowprec.to_bf16(f) for f in fs])).real.min() + 0.01
    assert np.isclose(lowprec.min_eig_rounded(fs, 0.01, lowprec.to_bf16), lam, rtol=1e-9, atol=1e-12)
