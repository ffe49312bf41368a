"""Exact (direct) solves of A X = B in float64.

Two independent routes to the unique solution x = A^{-1} b of an SPD
system, used to pin the iterative solvers:

* dense Cholesky of the materialised operator (the dense base case that
  Sec. 3.2 contrasts with iterative solves), via LAPACK potrf/potrs;
* the Kronecker eigendecomposition rule of App. A: Eigs(A (x) B) =
  Lambda_A (x) Lambda_B with eigenvectors V_A (x) V_B, combined with the
  spectral-function rule of App. A "Derived functions"
  (f(A) = V f(Lambda) V^T for symmetric PSD A) with f(t) = 1 / (t + sigma2).
  This covers one Kronecker term plus sigma2 I at any size.

TEST INFRASTRUCTURE: see the package docstring.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import kron


def cholesky_solve(terms, B: np.ndarray, sigma2: float = 0.0, diag=None) -> np.ndarray:
    """x = A^{-1} b for every row b of B, by dense Cholesky (small n)."""
    A = kron.dense_operator(terms, sigma2, diag)
    c = scipy.linalg.cho_factor(A, lower=True)
    return scipy.linalg.cho_solve(c, np.asarray(B, dtype=np.float64).T).T


def kron_eigs(factors):
    """Per-factor symmetric eigendecompositions (eigenvalues, eigenvectors)."""
    out = []
    for f in factors:
        f = np.asarray(f, dtype=np.float64)
        w, v = np.linalg.eigh(0.5 * (f + f.T))
        out.append((w, v))
    return out


def kron_eigenvalues(factors) -> np.ndarray:
    """Eigenvalues of K1 (x) K2 (x) ... as the Kronecker product of factor spectra (App. A)."""
    lam = np.array([1.0])
    for w, _ in kron_eigs(factors):
        lam = np.kron(lam, w)
    return lam


def kron_eig_solve(factors, B: np.ndarray, sigma2: float) -> np.ndarray:
    """x = (K1 (x) ... (x) KF + sigma2 I)^{-1} b for each row b, at any n.

    With K_k = Q_k L_k Q_k^T, the operator is (Q1 (x) ... ) diag(l1 (x) ... + sigma2)
    (Q1 (x) ...)^T, so the solve is a Kronecker MVM with the Q_k^T, a
    division by the shifted eigenvalue products, and a Kronecker MVM with
    the Q_k.
    """
    eig = kron_eigs(factors)
    qs = [v for _, v in eig]
    lam = np.array([1.0])
    for w, _ in eig:
        lam = np.kron(lam, w)
    C = kron.kron_apply([q.T for q in qs], B)
    C = C / (lam[None, :] + sigma2)
    return kron.kron_apply(qs, C)


def condition_number(factors, sigma2: float) -> float:
    """kappa(K1 (x) ... + sigma2 I) from the extreme eigenvalue products."""
    lam = kron_eigenvalues(factors) + sigma2
    return float(lam.max() / lam.min())


def solve(system_terms, B, sigma2=0.0, diag=None, dense_limit: int = 4096):
    """Exact solve by the cheapest exact route available for this operator."""
    n = kron.n_of(system_terms)
    if len(system_terms) == 1 and diag is None:
        return kron_eig_solve(system_terms[0], B, sigma2)
    if n <= dense_limit:
        return cholesky_solve(system_terms, B, sigma2, diag)
    raise ValueError("no exact route: use oracle.cg with a tight tolerance")
