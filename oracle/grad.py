"""Gradients of x = A^{-1} b through the operator's parameters, in float64.

App. B.2 gives the solve VJP (autograd rule 1): for y = Solve(A, b),
w^T dy/dtheta = -(A^{-1} w)^T (d_theta A_theta) (A^{-1} b), where theta is
the flattened list of the operator's differentiable arguments (the
flatten/unflatten construction of App. B.2).  With a loss L and its
cotangent g = dL/dx, lambda = A^{-T} g = A^{-1} g (A is symmetric; the
transpose rules of App. A give (A (x) B)^T = A^T (x) B^T), and

    dL/dtheta = - sum_r lambda_r^T (d A / d theta) x_r,     dL/db = lambda.

The printed form of the general recipe in App. B.2 drops the minus sign
that rule 1 carries; this oracle follows rule 1 (d(A^{-1}) = -A^{-1} dA A^{-1}).

Three independent routes are provided so each pins the others:
  grad_dense   : dense dL/dA = -sum_r lambda_r x_r^T, then the chain rule
                 through A = sum_j kron(...) + diag(d) + sigma2 I by
                 reshaping and summing (small n);
  grad_kron    : closed-form factor contractions at any n;
  grad_fd      : central finite differences of L with dense LU solves.

Gradients of a factor are entry-wise and unsymmetrised (each entry of the
stored factor is its own parameter).

TEST INFRASTRUCTURE: see the package docstring.
"""
from __future__ import annotations

import string

import numpy as np

from . import kron


def grad_dense(terms, X: np.ndarray, Lam: np.ndarray, diag_present: bool = False):
    """Chain rule from the dense gradient G_A = -sum_r lambda_r x_r^T.

    For factor k of term j, dL/dK_jk[a, i] sums G_A[p, q] * prod_{m != k}
    K_jm[p_m, q_m] over all row/column multi-indices p, q whose mode-k
    indices are a and i.  Returns (dfactors, dd or None, dsigma2).
    """
    X = np.asarray(X, dtype=np.float64)
    Lam = np.asarray(Lam, dtype=np.float64)
    dims = kron.dims_of(terms)
    F = len(dims)
    GA = -(Lam.T @ X)
    Gt = GA.reshape(dims + dims)
    letters = string.ascii_lowercase
    row = letters[:F]
    col = letters[F:2 * F]
    dfac = []
    for fs in terms:
        row_j = []
        for k in range(F):
            operands = [Gt]
            subs = [row + col]
            for m in range(F):
                if m != k:
                    operands.append(np.asarray(fs[m], dtype=np.float64))
                    subs.append(row[m] + col[m])
            expr = ",".join(subs) + "->" + row[k] + col[k]
            row_j.append(np.einsum(expr, *operands, optimize=True))
        dfac.append(row_j)
    dd = np.diag(GA).copy() if diag_present else None
    dsigma2 = float(np.trace(GA))
    return dfac, dd, dsigma2


def grad_kron(terms, X: np.ndarray, Lam: np.ndarray, diag_present: bool = False):
    """Closed-form factor gradients: dK_jk = -sum_r Lam_r,(k) Z_r,(k)^T.

    Z_r is x_r with every mode except k multiplied by that term's factor,
    and M_(k) is the mode-k unfolding (mode k first, the rest flattened).
    Two-factor row-major case: dK1 = -Lam K2 X^T, dK2 = -Lam^T K1 X.
    dd = -sum_r lambda_r * x_r (elementwise), dsigma2 = -sum_r lambda_r . x_r.
    """
    X = np.asarray(X, dtype=np.float64)
    Lam = np.asarray(Lam, dtype=np.float64)
    nrhs = X.shape[0]
    dims = kron.dims_of(terms)
    F = len(dims)
    dfac = []
    for fs in terms:
        row_j = []
        for k in range(F):
            T = X.reshape((nrhs,) + dims)
            for m in range(F):
                if m == k:
                    continue
                T = np.tensordot(np.asarray(fs[m], dtype=np.float64), T, axes=([1], [m + 1]))
                T = np.moveaxis(T, 0, m + 1)
            Zk = np.moveaxis(T, k + 1, 1).reshape(nrhs, dims[k], -1)
            Lk = np.moveaxis(Lam.reshape((nrhs,) + dims), k + 1, 1).reshape(nrhs, dims[k], -1)
            row_j.append(-np.einsum("rap,rip->ai", Lk, Zk, optimize=True))
        dfac.append(row_j)
    dd = -(Lam * X).sum(axis=0) if diag_present else None
    dsigma2 = float(-(Lam * X).sum())
    return dfac, dd, dsigma2


def loss(X: np.ndarray, W: np.ndarray) -> float:
    """L = sum_r w_r^T x_r (the linear loss of the gradient workloads)."""
    return float((np.asarray(X) * np.asarray(W)).sum())


def _dense_solve_loss(terms, sigma2, diag, B, W):
    A = kron.dense_operator(terms, sigma2, diag)
    X = np.linalg.solve(A, np.asarray(B, dtype=np.float64).T).T
    return loss(X, W)


def grad_fd(terms, sigma2, diag, B, W, which, h_rel: float = 1e-5) -> float:
    """Central finite difference of L = sum w^T A^{-1} b in one parameter.

    which = ("factor", j, k, a, i) | ("diag", p) | ("sigma2",).  A single
    factor entry is perturbed on its own, so A is no longer symmetric and
    the perturbed systems are solved with dense LU.
    """
    def perturbed(delta):
        t2 = [[np.array(f, dtype=np.float64, copy=True) for f in fs] for fs in terms]
        s2 = float(sigma2)
        d2 = None if diag is None else np.array(diag, dtype=np.float64, copy=True)
        if which[0] == "factor":
            _, j, k, a, i = which
            t2[j][k][a, i] += delta
        elif which[0] == "diag":
            d2[which[1]] += delta
        elif which[0] == "sigma2":
            s2 += delta
        else:
            raise ValueError(which)
        return _dense_solve_loss(t2, s2, d2, B, W)

    if which[0] == "factor":
        base = abs(terms[which[1]][which[2]][which[3], which[4]])
    elif which[0] == "diag":
        base = abs(diag[which[1]])
    else:
        base = abs(sigma2)
    h = h_rel * max(1.0, base)
    return (perturbed(h) - perturbed(-h)) / (2.0 * h)


def rbf_lengthscale_grad(dK: np.ndarray, K: np.ndarray, points: np.ndarray, ell: float) -> float:
    """Chain rule dL/dl = sum_{a,i} dL/dK[a,i] * K[a,i] (x_a - x_i)^2 / l^3 for the RBF factor."""
    p = np.asarray(points, dtype=np.float64)
    d2 = (p[:, None] - p[None, :]) ** 2
    return float((np.asarray(dK) * np.asarray(K) * d2).sum() / ell ** 3)
