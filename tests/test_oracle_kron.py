"""Pins for the oracle's operator and MVM (CPU only)."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import exact_ref as ex
from oracle import kron, direct

GOLD = os.path.join(os.path.dirname(__file__), "golden", "kron_worked_2x2.json")


def _rand_terms(rng, dims, nterms, symmetric=False):
    out = []
    for _ in range(nterms):
        row = []
        for m in dims:
            f = rng.standard_normal((m, m))
            if symmetric:
                f = f + f.T
            row.append(f)
        out.append(row)
    return out


def test_golden_worked_example_symmetric():
    g = json.load(open(GOLD))["symmetric"]
    K1, K2 = np.array(g["K1"], float), np.array(g["K2"], float)
    terms = [[K1, K2]]
    A = kron.dense_operator(terms, g["sigma2"])
    assert np.array_equal(A, np.array(g["dense_A"], float))
    y = kron.mvm(terms, np.array([g["x"]], float), g["sigma2"])
    assert np.array_equal(y[0], np.array(g["Ax"], float))
    assert np.array_equal(kron.operator_diagonal(terms, g["sigma2"]), np.array(g["diag_A"], float))
    lam = np.sort(direct.kron_eigenvalues(terms[0]) + g["sigma2"])
    assert np.allclose(lam, g["eigenvalues_sorted"], rtol=0, atol=1e-13)
    x = direct.cholesky_solve(terms, np.ones((1, 4)), g["sigma2"])
    assert np.allclose(x[0], g["b_ones_solution"], rtol=0, atol=1e-15)
    x2 = direct.kron_eig_solve(terms[0], np.ones((1, 4)), g["sigma2"])
    assert np.allclose(x2[0], g["b_ones_solution"], rtol=0, atol=1e-15)


def test_golden_worked_example_nonsymmetric_row_major():
    g = json.load(open(GOLD))["nonsymmetric"]
    terms = [[np.array(g["K1"], float), np.array(g["K2"], float)]]
    y = kron.mvm(terms, np.array([g["x"]], float))
    assert np.array_equal(y[0], np.array(g["Ax"], float))


@pytest.mark.parametrize("dims", [(2, 3), (3, 2, 2), (1, 4), (2, 1, 3), (5,)])
def test_mvm_matches_exact_kron_definition(dims):
    rng = np.random.default_rng(11)
    ints = [rng.integers(-3, 4, size=(m, m)) for m in dims]
    x = rng.integers(-5, 6, size=int(np.prod(dims)))
    # exact: Kronecker product by its entry definition, in rationals
    K = [[Fraction(1)]]
    for f in ints:
        K = ex.kron(K, ex.frac_matrix(f.tolist()))
    y_exact = ex.matvec(K, [Fraction(int(v)) for v in x])
    y = kron.mvm([[f.astype(float) for f in ints]], x[None, :].astype(float), sigma2=0.0)
    assert [Fraction(v) for v in y[0]] == y_exact     # integer data: float64 is exact here


@pytest.mark.parametrize("dims,nterms", [((3, 4), 1), ((2, 3, 5), 1), ((3, 3), 3), ((2, 2, 3), 2), ((7,), 2)])
def test_mvm_matches_numpy_kron_dense(dims, nterms):
    rng = np.random.default_rng(12)
    terms = _rand_terms(rng, dims, nterms)             # non-symmetric: catches transposed operands
    n = int(np.prod(dims))
    d = rng.uniform(0.1, 1.0, n)
    X = rng.standard_normal((3, n))
    dense = kron.dense_operator(terms, 0.3, d)
    y = kron.mvm(terms, X, 0.3, d)
    assert np.allclose(y, X @ dense.T, rtol=1e-13, atol=1e-13)


def test_dense_by_unit_vector_mvms():
    # Sec. 3.1: the dense matrix is MVM(e_1), ..., MVM(e_N)
    rng = np.random.default_rng(13)
    terms = _rand_terms(rng, (2, 3, 2), 2)
    n = 12
    cols = kron.mvm(terms, np.eye(n), 0.5)             # row i of the result is A e_i
    assert np.allclose(cols.T, kron.dense_operator(terms, 0.5), rtol=0, atol=1e-13)


def test_identity_and_diagonal_factors():
    rng = np.random.default_rng(14)
    x = rng.standard_normal((2, 24))
    y = kron.mvm([[np.eye(2), np.eye(3), np.eye(4)]], x, sigma2=0.25)
    assert np.allclose(y, 1.25 * x, rtol=0, atol=1e-15)
    a, b, c = rng.standard_normal(2), rng.standard_normal(3), rng.standard_normal(4)
    y = kron.mvm([[np.diag(a), np.diag(b), np.diag(c)]], x)
    scale = (a[:, None, None] * b[None, :, None] * c[None, None, :]).reshape(-1)
    assert np.allclose(y, x * scale[None, :], rtol=1e-14, atol=1e-14)


def test_kron_diagonal_rule_pins_row_major():
    rng = np.random.default_rng(15)
    fs = [rng.standard_normal((m, m)) for m in (2, 3, 4)]
    assert np.allclose(kron.kron_diagonal(fs), np.diag(kron.dense_kron(fs)), rtol=0, atol=1e-14)
    # the column-major reading would reverse the order of the factors
    rev = kron.dense_kron(fs[::-1])
    assert not np.allclose(kron.kron_diagonal(fs), np.diag(rev))


def test_transpose_rule():
    # App. A: (A (x) B)^T = A^T (x) B^T
    rng = np.random.default_rng(16)
    fs = [rng.standard_normal((m, m)) for m in (3, 4)]
    x = rng.standard_normal((1, 12))
    y = kron.mvm([[f.T for f in fs]], x)
    assert np.allclose(y[0], kron.dense_kron(fs).T @ x[0], rtol=1e-13, atol=1e-13)


def test_mvm_entry_matches_full_mvm():
    rng = np.random.default_rng(17)
    terms = _rand_terms(rng, (3, 4, 5), 2)
    d = rng.uniform(0.1, 1, 60)
    x = rng.standard_normal(60)
    y = kron.mvm(terms, x[None], 0.2, d)[0]
    for idx in (0, 7, 31, 59):
        assert np.isclose(kron.mvm_entry(terms, x, idx, 0.2, d), y[idx], rtol=1e-13, atol=1e-13)


def test_relres_zero_for_exact_solution():
    rng = np.random.default_rng(18)
    fs = [np.eye(3) * 2.0, np.eye(2) * 3.0]
    B = rng.standard_normal((2, 6))
    X = B / 7.0
    assert np.all(kron.relres([fs], X, B, sigma2=1.0) < 1e-15)
