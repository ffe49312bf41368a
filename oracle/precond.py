"""Operator diagonals, diagonal estimators and preconditioned CG, in numpy float64.

The paper's Diag rules (App. A, "Diagonal"): Diag(A + B) = Diag(A) + Diag(B) and
Diag(A (x) B) = vec(Diag(A) Diag(B)^T) (row-major vec here), so the diagonal of
a sum of Kronecker terms plus a diagonal is exact at O(n) cost
(kron.operator_diagonal).  Where no rule applies the paper estimates it from
MVMs with probes (Sec. 3.3, "stochastic diagonal and trace estimation"):

* Hutchinson:             Diag(A) ~ (1/N) sum_j z_j . A z_j  (. is elementwise),
  with probes of identity covariance shared by every term of a Sum;
* doubly stochastic (App. B.1): for A = sum_i A_i,
                          Diag(A) ~ (1/N) sum_j sum_i z_ij . A_i z_ij,
  a fresh probe for every term, whose variance per entry is the sum of the
  terms' variances instead of the variance of the sum (App. B.1 derives the
  trace case; the diagonal follows the same steps).

Per-entry variance of one probe's z . A z (a short derivation): entry k is
sum_l A_kl z_k z_l, so with Gaussian z it is A_kk^2 + sum_l A_kl^2, and with
Rademacher z (z_k^2 = 1) it is sum over l != k of A_kl^2.

Preconditioned CG: the paper pairs CG and GMRES with preconditioners in its
applications (Sec. 3.2, Sec. 3.3 and the sum-structure experiments of App. D.3)
but prints no steps, so this is the textbook recurrence (Saad, Iterative Methods, Alg. 9.1)
with x0 = 0 and a symmetric positive definite M:

    r0 = b, z0 = M^{-1} r0, p0 = z0, rho0 = r0.z0
    repeat:  q = A p;  alpha = rho / p.q;  x += alpha p;  r -= alpha q
             stop when ||r|| <= tol ||b||
             z = M^{-1} r;  rho' = r.z;  beta = rho' / rho;  p = z + beta p

Two preconditioners are built from the operator's structure:
* Jacobi, M = Diag(A), from the exact Kronecker diagonal rule;
* Kronecker-eigen, M = (first Kronecker term) + c I, applied exactly by the
  Kronecker eigendecomposition (App. A, as in direct.kron_eig_solve), with the
  shift c = Tr(A - first term) / n = sigma2 + mean(d) + sum over the other
  terms of the product of their factors' mean diagonals (Tr(K1 (x) K2) =
  Tr(K1) Tr(K2)).  For one term plus sigma2 I, M = A.
Readings where the paper is silent: the preconditioners, the trace-matching
shift, and stopping on the unpreconditioned residual as plain CG does.

TEST INFRASTRUCTURE: see the package docstring.
"""
from __future__ import annotations

from typing import Callable, List, Sequence, Tuple

import numpy as np

from . import direct, kron


def pcg(apply_A: Callable[[np.ndarray], np.ndarray], apply_Minv: Callable[[np.ndarray], np.ndarray],
        B: np.ndarray, tol: float, max_iters: int) -> Tuple[np.ndarray, np.ndarray, List[str]]:
    """Preconditioned CG on each row of B (shape (nrhs, n)); returns X, iterations, statuses
    ("ok", "not_converged", "not_spd", "nonfinite")."""
    B = np.asarray(B, dtype=np.float64)
    X = np.zeros_like(B)
    iters = np.zeros(B.shape[0], dtype=np.int64)
    status = []
    for g, b in enumerate(B):
        bn = float(np.linalg.norm(b))
        if not np.isfinite(bn):
            status.append("nonfinite")
            continue
        x = np.zeros_like(b)
        r = b.copy()
        if bn == 0.0:
            status.append("ok")
            continue
        z = apply_Minv(r[None, :])[0]
        rho = float(r @ z)
        if not (np.isfinite(rho) and rho > 0.0):
            status.append("not_spd")
            continue
        p = z.copy()
        st = "not_converged"
        k = 0
        while k < max_iters:
            q = apply_A(p[None, :])[0]
            mu = float(p @ q)
            if not (np.isfinite(mu) and mu > 0.0):
                st = "not_spd"
                break
            alpha = rho / mu
            x = x + alpha * p
            r = r - alpha * q
            k += 1
            rr = float(r @ r)
            if not np.isfinite(rr):
                st = "nonfinite"
                break
            if np.sqrt(rr) <= tol * bn:
                st = "ok"
                break
            z = apply_Minv(r[None, :])[0]
            rho_new = float(r @ z)
            if not (np.isfinite(rho_new) and rho_new > 0.0):
                st = "not_spd"
                break
            p = z + (rho_new / rho) * p
            rho = rho_new
        X[g] = x
        iters[g] = k
        status.append(st)
    return X, iters, status


def jacobi_inverse(terms, sigma2: float = 0.0, diag=None) -> np.ndarray:
    """1 / Diag(A) by the exact Sum and Kronecker diagonal rules."""
    return 1.0 / kron.operator_diagonal(terms, sigma2, diag)


def kron_eig_shift(terms, sigma2: float = 0.0, diag=None) -> float:
    """c = Tr(A - first Kronecker term) / n."""
    c = float(sigma2)
    if diag is not None:
        c += float(np.mean(np.asarray(diag, dtype=np.float64)))
    for fs in terms[1:]:
        c += float(np.prod([np.mean(np.diag(np.asarray(f, dtype=np.float64))) for f in fs]))
    return c


def kron_eig_preconditioner(terms, sigma2: float = 0.0, diag=None) -> Callable[[np.ndarray], np.ndarray]:
    """R -> (first term + c I)^{-1} R by the Kronecker eigen rules."""
    facs = [np.asarray(f, dtype=np.float64) for f in terms[0]]
    c = kron_eig_shift(terms, sigma2, diag)
    return lambda R: direct.kron_eig_solve(facs, R, c)


def hutchinson_diagonal(apply_A: Callable[[np.ndarray], np.ndarray], Z: np.ndarray) -> np.ndarray:
    """(1/N) sum_j z_j . A z_j over the rows of Z (shape (N, n))."""
    Z = np.asarray(Z, dtype=np.float64)
    return (Z * apply_A(Z)).mean(axis=0)


def doubly_stochastic_diagonal(apply_terms: Sequence[Callable[[np.ndarray], np.ndarray]],
                               Zs: Sequence[np.ndarray]) -> np.ndarray:
    """(1/N) sum_j sum_i z_ij . A_i z_ij: term i uses its own probe rows Zs[i] (shape (N, n))."""
    out = 0.0
    for apply_i, Z in zip(apply_terms, Zs):
        Z = np.asarray(Z, dtype=np.float64)
        out = out + (Z * apply_i(Z)).mean(axis=0)
    return out


def probe_variance(A: np.ndarray, kind: str = "rademacher") -> np.ndarray:
    """Per-entry variance of z . A z for one probe z with i.i.d. entries (dense A, small n)."""
    A = np.asarray(A, dtype=np.float64)
    a2 = (A * A).sum(axis=1)                       # sum_l A_kl^2
    d = np.diag(A)
    if kind == "rademacher":
        return a2 - d * d
    if kind == "gaussian":
        return a2 + d * d
    raise ValueError(kind)
