"""Log-determinant by stochastic Lanczos quadrature (SLQ), in numpy float64.

The paper defines LogDet(A) = Tr(Log(A)) with Log(A) = V log(Lambda) V^T for
a symmetric PSD operator (App. A "Derived functions"), and lists stochastic
Lanczos quadrature as the base-case iterative algorithm for f(A) of a
self-adjoint operator (App. C, table of base-case iterative methods); GP
training needs log|K| and its gradient (Sec. 4, Gaussian processes).  The
paper prints no SLQ steps, so this is the textbook method:

* Hutchinson: Tr(f(A)) = E[z^T f(A) z] for probes with E[z z^T] = I
  (Rademacher entries here);
* Lanczos quadrature: m Lanczos steps from v1 = z / ||z|| give a symmetric
  tridiagonal T_m, and z^T f(A) z ~= ||z||^2 e1^T f(T_m) e1
  = ||z||^2 sum_k tau_k^2 f(theta_k)   (theta_k, tau_k: eigenvalues of T_m
  and first components of its normalised eigenvectors: Gauss quadrature);
* the Lanczos coefficients of the Krylov space of z are available from a CG
  solve of A x = z (the CG-Lanczos relation, Saad, Iterative Methods,
  Sec. 6.7.3): with CG step lengths alpha_j and ratios beta_j =
  rho_{j+1} / rho_j,
      T[0, 0] = 1 / alpha_0,
      T[j, j] = 1 / alpha_j + beta_{j-1} / alpha_{j-1}          (j >= 1),
      T[j, j+1] = T[j+1, j] = sqrt(beta_j) / alpha_j,
  so one batched CG over the probes gives both A^{-1} Z and the quadrature.

The gradient d log|A| / d theta = Tr(A^{-1} dA/dtheta) is estimated by the
same probes as mean_z (A^{-1} z)^T (dA/dtheta) z, i.e. the solve VJP of
App. B.2 evaluated with X = Z and Lambda = A^{-1} Z (up to its sign).

Readings where the paper is silent: Rademacher probes; the quadrature uses
the coefficients of the CG iterations actually run (fewer than m when a
probe's CG converges, which leaves the Krylov space nearly invariant).

TEST INFRASTRUCTURE: see the package docstring.
"""
from __future__ import annotations

from typing import Callable, Tuple

import numpy as np
import scipy.linalg

from . import direct


def lanczos(apply_A: Callable[[np.ndarray], np.ndarray], b: np.ndarray, m: int) -> Tuple[np.ndarray, np.ndarray]:
    """m steps of Lanczos from b / ||b|| with full reorthogonalisation.

    Returns the diagonal (length k) and off-diagonal (length k - 1) of the
    tridiagonal T_k, k <= m (fewer when the Krylov space becomes invariant).
    """
    b = np.asarray(b, dtype=np.float64)
    V = [b / np.linalg.norm(b)]
    diag, off = [], []
    for j in range(m):
        w = apply_A(V[j][None, :])[0]
        a = float(V[j] @ w)
        diag.append(a)
        for v in V:                       # full reorthogonalisation (twice is enough)
            w = w - (v @ w) * v
        for v in V:
            w = w - (v @ w) * v
        nb = float(np.linalg.norm(w))
        if j == m - 1 or nb <= 1e-12 * abs(a):
            break
        off.append(nb)
        V.append(w / nb)
    return np.array(diag), np.array(off)


def cg_coefficients(apply_A: Callable[[np.ndarray], np.ndarray], b: np.ndarray, m: int,
                    tol: float = 0.0) -> Tuple[np.ndarray, np.ndarray]:
    """Textbook CG on A x = b (x0 = 0) for at most m iterations, stopping when
    ||r|| <= tol ||b||; returns the step lengths alpha_j and ratios beta_j."""
    b = np.asarray(b, dtype=np.float64)
    r = b.copy()
    p = r.copy()
    rho = float(r @ r)
    stop = tol * np.sqrt(rho)
    alphas, betas = [], []
    for _ in range(m):
        q = apply_A(p[None, :])[0]
        alpha = rho / float(p @ q)
        r = r - alpha * q
        rho_new = float(r @ r)
        beta = rho_new / rho
        alphas.append(alpha)
        betas.append(beta)
        if np.sqrt(rho_new) <= stop:
            break
        p = r + beta * p
        rho = rho_new
    return np.array(alphas), np.array(betas)


def tridiagonal_from_cg(alphas: np.ndarray, betas: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Lanczos tridiagonal (diagonal, off-diagonal) of k CG iterations."""
    k = len(alphas)
    d = np.empty(k)
    d[0] = 1.0 / alphas[0]
    for j in range(1, k):
        d[j] = 1.0 / alphas[j] + betas[j - 1] / alphas[j - 1]
    e = np.sqrt(betas[:k - 1]) / alphas[:k - 1]
    return d, e


def quadrature(d: np.ndarray, e: np.ndarray, f: Callable[[np.ndarray], np.ndarray]) -> float:
    """e1^T f(T) e1 for the symmetric tridiagonal T (Gauss quadrature nodes and weights)."""
    if len(d) == 1:
        return float(f(np.array([d[0]]))[0])
    theta, S = scipy.linalg.eigh_tridiagonal(d, e)
    return float(np.sum(S[0, :] ** 2 * f(theta)))


def probe_logdets(apply_A: Callable[[np.ndarray], np.ndarray], Z: np.ndarray, m: int,
                  tol: float = 0.0) -> np.ndarray:
    """Per-probe estimates ||z||^2 e1^T log(T) e1 with T from the CG coefficients."""
    out = []
    for z in np.asarray(Z, dtype=np.float64):
        if not np.any(z):                 # z = 0: z^T log(A) z = 0 (no iteration runs)
            out.append(0.0)
            continue
        a, b = cg_coefficients(apply_A, z, m, tol)
        d, e = tridiagonal_from_cg(a, b)
        out.append(float(z @ z) * quadrature(d, e, np.log))
    return np.array(out)


def slq_logdet(apply_A: Callable[[np.ndarray], np.ndarray], Z: np.ndarray, m: int, tol: float = 0.0) -> float:
    """Mean of the per-probe estimates: the SLQ estimate of log det A."""
    return float(np.mean(probe_logdets(apply_A, Z, m, tol)))


def kron_logdet(factors, sigma2: float) -> float:
    """log det (K1 (x) ... (x) KF + sigma2 I) = sum of log(eigenvalue products + sigma2) (App. A)."""
    return float(np.sum(np.log(direct.kron_eigenvalues(factors) + sigma2)))


def kron_trace_inverse(factors, sigma2: float) -> float:
    """Tr (K1 (x) ... + sigma2 I)^{-1} = d log det / d sigma2, from the Kronecker spectrum."""
    return float(np.sum(1.0 / (direct.kron_eigenvalues(factors) + sigma2)))
