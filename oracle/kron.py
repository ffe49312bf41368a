"""Operator A = sum_j (K_j1 (x) ... (x) K_jF) + diag(d) + sigma2 I, in float64.

Sec. 3.1 defines a linear operator by its MVM; the Dense operator's MVM is
the ordinary matrix product and the Diagonal operator's MVM is d_i v_i.
Sec. 3.2 composes operators: the Sum's MVM is the sum of the children's
MVMs, and a Kronecker product is applied without forming it, at cost
tau_A N_B + N_A tau_B (Table 2).  Row-major vec: the Kronecker product acts
on X = x.reshape(n1, ..., nF) by multiplying each mode by its factor.

TEST INFRASTRUCTURE: see the package docstring.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


def dims_of(terms) -> tuple:
    return tuple(int(f.shape[0]) for f in terms[0])


def n_of(terms) -> int:
    return int(np.prod(dims_of(terms)))


def dense_kron(factors: Sequence[np.ndarray]) -> np.ndarray:
    """Dense K_1 (x) K_2 (x) ... via numpy.kron (library primitive)."""
    out = np.array([[1.0]])
    for f in factors:
        out = np.kron(out, np.asarray(f, dtype=np.float64))
    return out


def dense_operator(terms, sigma2: float = 0.0, diag=None) -> np.ndarray:
    """Dense A = sum_j kron(terms[j]) + diag(d) + sigma2 I (small n only)."""
    a = None
    for fs in terms:
        k = dense_kron(fs)
        a = k if a is None else a + k
    n = a.shape[0]
    a = a.copy()
    a[np.diag_indices(n)] += sigma2
    if diag is not None:
        a[np.diag_indices(n)] += np.asarray(diag, dtype=np.float64)
    return a


def kron_apply(factors: Sequence[np.ndarray], X: np.ndarray) -> np.ndarray:
    """Apply one Kronecker term to each row of X (shape (nrhs, n)).

    Each factor multiplies its own mode of the tensor X.reshape(nrhs, n1..nF):
    Y[r, a, b, c] = sum_{i,j,k} K1[a,i] K2[b,j] K3[c,k] X[r, i, j, k].
    Done one mode at a time with numpy.tensordot (a matmul), which is the
    mode-wise evaluation whose cost Table 2 states.
    """
    X = np.asarray(X, dtype=np.float64)
    nrhs = X.shape[0]
    dims = tuple(int(f.shape[0]) for f in factors)
    T = X.reshape((nrhs,) + dims)
    for k, f in enumerate(factors):
        # contract factor columns with tensor mode k+1, put the new axis back in place
        T = np.tensordot(np.asarray(f, dtype=np.float64), T, axes=([1], [k + 1]))
        T = np.moveaxis(T, 0, k + 1)
    return T.reshape(nrhs, -1)


def mvm(terms, X: np.ndarray, sigma2: float = 0.0, diag=None) -> np.ndarray:
    """A X for every row of X: Sum composition of Kronecker terms and the diagonal."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.zeros_like(X)
    for fs in terms:
        Y += kron_apply(fs, X)
    if sigma2:
        Y += sigma2 * X
    if diag is not None:
        Y += np.asarray(diag, dtype=np.float64)[None, :] * X
    return Y


def mvm_entry(terms, x: np.ndarray, index: int, sigma2: float = 0.0, diag=None) -> float:
    """One output entry (A x)[index] for a single vector x, by its definition.

    Used to spot-check full-size GPU products: for the row-major multi-index
    (a, b, c) of ``index``, sum_j sum_{i,j,k} K1[a,i] K2[b,j] K3[c,k] x[i,j,k].
    Cost O(n) per entry.
    """
    dims = dims_of(terms)
    multi = np.unravel_index(index, dims)
    T = np.asarray(x, dtype=np.float64).reshape(dims)
    total = 0.0
    for fs in terms:
        v = T
        for f, a in zip(fs, multi):
            # contract the leading remaining mode with row a of this factor
            v = np.tensordot(np.asarray(f, dtype=np.float64)[a], v, axes=([0], [0]))
        total += float(v)
    d_add = sigma2
    if diag is not None:
        d_add = d_add + float(diag[index])
    return total + d_add * float(np.asarray(x).reshape(-1)[index])


def kron_diagonal(factors: Sequence[np.ndarray]) -> np.ndarray:
    """Diag(K1 (x) K2 (x) ...) by the App. A rule Diag(A (x) B) = vec(Diag(A) Diag(B)^T).

    Applied recursively; vec is row-major, so the outer product's rows are
    indexed by the first factor.
    """
    out = np.array([1.0])
    for f in factors:
        out = np.outer(out, np.diag(np.asarray(f, dtype=np.float64))).reshape(-1)
    return out


def operator_diagonal(terms, sigma2: float = 0.0, diag=None) -> np.ndarray:
    """Diag(A) by the Sum rule Diag(A + B) = Diag(A) + Diag(B) (App. A)."""
    out = sum(kron_diagonal(fs) for fs in terms)
    out = out + sigma2
    if diag is not None:
        out = out + np.asarray(diag, dtype=np.float64)
    return out


def relres(terms, X: np.ndarray, B: np.ndarray, sigma2: float = 0.0, diag=None) -> np.ndarray:
    """True relative residual ||b - A x|| / ||b|| per row, A applied in float64."""
    X = np.asarray(X, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    R = B - mvm(terms, X, sigma2, diag)
    bn = np.linalg.norm(B, axis=1)
    rn = np.linalg.norm(R, axis=1)
    return np.where(bn > 0, rn / np.where(bn > 0, bn, 1.0), rn)
