"""Conjugate gradients and float64-residual iterative refinement, in numpy.

The paper's base case for solves with a PSD operator is conjugate gradients
(Sec. 3.2 "Decoration/annotation operators": solve[PSD] uses CG; App. C
table of base-case iterative methods).  It prints no CG steps and refers to
the standard texts, so this is the textbook Hestenes-Stiefel recurrence
with x0 = 0:

    r0 = b, p0 = r0, rho0 = r0.r0
    repeat:  q = A p;  mu = p.q;  alpha = rho / mu
             x += alpha p;  r -= alpha q;  rho' = r.r
             stop when sqrt(rho') <= tol * ||b||
             beta = rho' / rho;  p = r + beta p

Several right-hand sides are independent CG runs advanced together; a
column that has converged is frozen, and the solve ends when every column
has converged, as in the multi-RHS block solves of App. D.5 (stopping on
the convergence of all solves, not their mean).

Readings where the paper is silent: "tolerance" is the relative residual
||b - A x|| / ||b|| per right-hand side; a non-positive or non-finite p.Ap
is a breakdown ("not_spd"); non-finite input gives "nonfinite"; b = 0 gives
x = 0 after zero iterations.

TEST INFRASTRUCTURE: see the package docstring.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

OK = "ok"
NOT_CONVERGED = "not_converged"
STAGNATED = "stagnated"
NOT_SPD = "not_spd"
NONFINITE = "nonfinite"


@dataclass
class CGResult:
    X: np.ndarray
    iters: np.ndarray
    status: List[str]
    relres_recursive: np.ndarray
    history: Optional[dict] = None


def _round(v: np.ndarray, dtype) -> np.ndarray:
    if dtype is None or dtype == np.float64:
        return v
    return v.astype(dtype).astype(np.float64)


def cg(apply_A: Callable[[np.ndarray], np.ndarray], B: np.ndarray, tol: float,
       max_iters: int, dtype=None, keep_history: bool = False) -> CGResult:
    """Textbook CG on each row of B (shape (nrhs, n)).

    apply_A maps an (m, n) block of vectors to A times each row.  ``dtype``
    (e.g. numpy.float32) rounds the stored vectors x, r, p, q to that type
    after every update while the scalars and dot products stay float64; it
    emulates a low-precision working copy and is None for plain float64.
    """
    B = np.asarray(B, dtype=np.float64)
    nrhs, n = B.shape
    X = np.zeros_like(B)
    R = _round(B.copy(), dtype)
    P = R.copy()
    rho = np.einsum("ij,ij->i", R, R)
    bnorm = np.linalg.norm(B, axis=1)
    iters = np.zeros(nrhs, dtype=np.int64)
    status = [OK] * nrhs
    active = np.ones(nrhs, dtype=bool)
    for i in range(nrhs):
        if not np.all(np.isfinite(B[i])):
            status[i] = NONFINITE
            active[i] = False
        elif np.sqrt(rho[i]) <= tol * bnorm[i]:
            active[i] = False           # includes b = 0: x = 0, zero iterations
    hist = {"R": [R.copy()], "P": [P.copy()], "X": [X.copy()]} if keep_history else None
    for _ in range(max_iters):
        idx = np.nonzero(active)[0]
        if idx.size == 0:
            break
        Q = _round(apply_A(P[idx]), dtype)
        mu = np.einsum("ij,ij->i", P[idx], Q)
        bad = ~(np.isfinite(mu) & (mu > 0))
        for t, i in enumerate(idx):
            if bad[t]:
                status[i] = NOT_SPD if np.isfinite(mu[t]) else NONFINITE
                active[i] = False
        keep = ~bad
        idx, Q, mu = idx[keep], Q[keep], mu[keep]
        if idx.size == 0:
            continue
        alpha = rho[idx] / mu
        X[idx] = _round(X[idx] + alpha[:, None] * P[idx], dtype)
        R[idx] = _round(R[idx] - alpha[:, None] * Q, dtype)
        rho_new = np.einsum("ij,ij->i", R[idx], R[idx])
        iters[idx] += 1
        beta = rho_new / rho[idx]
        P[idx] = _round(R[idx] + beta[:, None] * P[idx], dtype)
        rho[idx] = rho_new
        done = np.sqrt(rho_new) <= tol * bnorm[idx]
        active[idx[done]] = False
        if keep_history:
            hist["R"].append(R.copy())
            hist["P"].append(P.copy())
            hist["X"].append(X.copy())
    for i in range(nrhs):
        if active[i]:
            status[i] = NOT_CONVERGED
    rel = np.sqrt(np.maximum(rho, 0.0)) / np.where(bnorm > 0, bnorm, 1.0)
    return CGResult(X, iters, status, rel, hist)


@dataclass
class RefineResult:
    X: np.ndarray
    sweeps: np.ndarray
    inner_iters: np.ndarray
    status: List[str]
    relres: np.ndarray
    relres_history: List[np.ndarray] = field(default_factory=list)


def refine(apply_A64: Callable, apply_A_low: Callable, B: np.ndarray, tol: float,
           inner_tol: float, max_sweeps: int, inner_max_iters: int,
           low_dtype=np.float32) -> RefineResult:
    """Iterative refinement with a float64 residual and a low-precision inner CG.

    The paper supports low precision by algorithmic modification (Sec. 3.4
    "Low precision linear algebra", App. C.3) but prints no scheme.  This is
    classical mixed-precision refinement: r = b - A x in float64; stop when
    ||r|| / ||b|| <= tol; otherwise solve A_low d = r / ||r|| with CG in
    the working precision to inner_tol and update x += ||r|| d in float64.
    A sweep that fails to halve ||r|| twice in a row ends the solve as
    "stagnated".  (The paper fixes no schedule.  This one is pinned by what
    mathematics fixes: float32 inner solves reach float64 accuracy, and an
    inconsistent inner operator makes it stagnate.)
    """
    B = np.asarray(B, dtype=np.float64)
    nrhs = B.shape[0]
    X = np.zeros_like(B)
    bnorm = np.linalg.norm(B, axis=1)
    sweeps = np.zeros(nrhs, dtype=np.int64)
    inner = np.zeros(nrhs, dtype=np.int64)
    status = [OK] * nrhs
    active = np.ones(nrhs, dtype=bool)
    prev = np.full(nrhs, np.inf)
    slow = np.zeros(nrhs, dtype=np.int64)
    hist = []
    rel = np.zeros(nrhs)
    for i in range(nrhs):
        if not np.all(np.isfinite(B[i])):
            status[i] = NONFINITE
            active[i] = False
    for s in range(max_sweeps + 1):
        R = B - apply_A64(X)
        rn = np.linalg.norm(R, axis=1)
        rel = np.where(bnorm > 0, rn / np.where(bnorm > 0, bnorm, 1.0), rn)
        hist.append(rel.copy())
        for i in range(nrhs):
            if not active[i]:
                continue
            if rel[i] <= tol:
                active[i] = False
                continue
            slow[i] = slow[i] + 1 if rn[i] > 0.5 * prev[i] else 0
            if slow[i] >= 2:
                status[i] = STAGNATED
                active[i] = False
        prev = rn
        idx = np.nonzero(active)[0]
        if idx.size == 0 or s == max_sweeps:
            break
        rhs = R[idx] / rn[idx, None]
        res = cg(apply_A_low, rhs, inner_tol, inner_max_iters, dtype=low_dtype)
        for t, i in enumerate(idx):
            if res.status[t] in (NOT_SPD, NONFINITE):
                status[i] = res.status[t]
                active[i] = False
        X[idx] = X[idx] + rn[idx, None] * res.X
        sweeps[idx] += 1
        inner[idx] += res.iters
    for i in range(nrhs):
        if active[i] and status[i] == OK and rel[i] > tol:
            status[i] = NOT_CONVERGED
    return RefineResult(X, sweeps, inner, status, rel, hist)


# Reliable updates: a recursive residual below this fraction of the last true residual is taken as
# the working precision's noise floor (the right-hand side waits for its update there).
NOISE_FLOOR = 1e-5


@dataclass
class ReliableResult:
    X: np.ndarray
    iters: np.ndarray
    updates: np.ndarray
    status: List[str]
    relres_true: np.ndarray
    relres_recursive: np.ndarray


def reliable(apply_A64: Callable, apply_A_low: Callable, B: np.ndarray, tol: float, delta: float,
             max_iters: int, check_every: int, low_dtype=np.float32, restart_dir: bool = False) -> ReliableResult:
    """One low-precision CG whose residual is replaced by the float64 true residual ("reliable
    updates"), the reading of the paper's low precision by algorithmic modification (Sec. 3.4,
    App. C.3) that the library builds; the paper prints no scheme, so this follows that reading:

    * the working vectors x_lo, r, p and the products q = A_low p are rounded to low_dtype after
      every update; the scalars alpha, beta, rho and every dot product are float64;
    * start: r = b (rounded), x = 0 (float64), x_lo = 0, p = 0, beta = 0, rho = r.r,
      ||b||^2 = rho, rmax = sqrt(rho);
    * each iteration of an active right-hand side: p = r + beta p, q = A_low p, alpha = rho / p.q,
      x_lo += alpha p, r -= alpha q, rho' = r.r; it stops (waits) when sqrt(rho') <= tol ||b||,
      or at max_iters (not converged); otherwise it asks for an update, and keeps iterating, once
      sqrt(rho') < delta rmax, unless sqrt(rho') < NOISE_FLOOR rmax, where it waits for the update
      (that far below the last true residual the working-precision recursion is rounding noise);
      then beta = rho' / rho, rho = rho';
    * the iterations run in chunks of check_every; after each chunk, every right-hand side that
      asked for an update (or waits after converging) gets one: x += x_lo in float64, x_lo = 0,
      r64 = b - A x in float64, r = r64 (rounded), rho_t = r64.r64; it is finished when
      sqrt(rho_t) <= tol ||b||; otherwise beta = rho_t beta / rho (0 with restart_dir: the
      direction restarts), rho = rho_t, rmax = sqrt(rho_t), and it runs again unless it hit
      max_iters or its recursive residual converged three updates in a row without the true
      residual following ("stagnated"; a wait at the noise floor is no convergence);
    * at the end, right-hand sides that stopped without a certified residual get a last fold and
      float64 residual.

    Columns are independent; a breakdown (p.q <= 0 or non-finite) stops a column as in cg().
    """
    B = np.asarray(B, dtype=np.float64)
    nrhs, n = B.shape
    X = np.zeros_like(B)
    xl = np.zeros_like(B)
    R = _round(B.copy(), low_dtype)
    P = np.zeros_like(B)
    rho = np.einsum("ij,ij->i", R, R)
    tol2 = tol * tol * rho
    beta = np.zeros(nrhs)
    rmax = np.sqrt(rho)
    iters = np.zeros(nrhs, dtype=np.int64)
    updates = np.zeros(nrhs, dtype=np.int64)
    fails = np.zeros(nrhs, dtype=np.int64)
    status: List[Optional[str]] = [None] * nrhs
    active = np.ones(nrhs, dtype=bool)
    need = np.zeros(nrhs, dtype=bool)
    rho_true = rho.copy()
    noise = np.zeros(nrhs, dtype=bool)
    for i in range(nrhs):
        if not np.all(np.isfinite(B[i])):
            status[i], active[i] = NONFINITE, False
        elif rho[i] <= tol2[i]:
            status[i], active[i] = OK, False       # includes b = 0
    while active.any():
        for _ in range(check_every):
            idx = np.nonzero(active)[0]
            if idx.size == 0:
                break
            P[idx] = _round(R[idx] + beta[idx, None] * P[idx], low_dtype)
            Q = _round(apply_A_low(P[idx]), low_dtype)
            mu = np.einsum("ij,ij->i", P[idx], Q)
            for t, i in enumerate(idx):
                if not (np.isfinite(mu[t]) and mu[t] > 0):
                    status[i] = NOT_SPD if np.isfinite(mu[t]) else NONFINITE
                    active[i] = False
            keep = np.array([active[i] for i in idx], dtype=bool)
            idx, Q, mu = idx[keep], Q[keep], mu[keep]
            if idx.size == 0:
                continue
            alpha = rho[idx] / mu
            xl[idx] = _round(xl[idx] + alpha[:, None] * P[idx], low_dtype)
            R[idx] = _round(R[idx] - alpha[:, None] * Q, low_dtype)
            rho_new = np.einsum("ij,ij->i", R[idx], R[idx])
            iters[idx] += 1
            for t, i in enumerate(idx):
                if not np.isfinite(rho_new[t]):
                    status[i], active[i] = NONFINITE, False
                elif rho_new[t] <= tol2[i]:
                    need[i], active[i] = True, False
                elif iters[i] >= max_iters:
                    status[i], active[i] = NOT_CONVERGED, False
                elif rho_new[t] < delta * delta * rmax[i] * rmax[i]:
                    need[i] = True
                    if rho_new[t] < NOISE_FLOOR * NOISE_FLOOR * rmax[i] * rmax[i]:
                        noise[i], active[i] = True, False
            beta[idx] = rho_new / rho[idx]
            rho[idx] = rho_new
        for i in np.nonzero(need)[0]:
            was_active = active[i]
            X[i] += xl[i]
            xl[i] = 0.0
            r64 = B[i] - apply_A64(X[i][None, :])[0]
            rt = float(r64 @ r64)
            R[i] = _round(r64, low_dtype)
            rho_true[i] = rt
            need[i] = False
            updates[i] += 1
            run = False
            if not np.isfinite(rt):
                status[i] = NONFINITE
            elif rt <= tol2[i]:
                status[i] = OK
            else:
                fails[i] = fails[i] + 1 if not (was_active or noise[i]) else 0
                if fails[i] >= 3:
                    status[i] = STAGNATED
                elif iters[i] >= max_iters:
                    status[i] = NOT_CONVERGED
                else:
                    run = True
                beta[i] = 0.0 if restart_dir else (rt * beta[i] / rho[i] if rho[i] > 0 else beta[i])
                rho[i] = rt
                rmax[i] = np.sqrt(rt)
            active[i] = run
            noise[i] = False
    for i in range(nrhs):
        if status[i] != OK and np.isfinite(B[i]).all():
            X[i] += xl[i]
            xl[i] = 0.0
            r64 = B[i] - apply_A64(X[i][None, :])[0]
            rho_true[i] = float(r64 @ r64)
        if status[i] is None:
            status[i] = NOT_CONVERGED
    bn2 = np.where(tol2 > 0, tol2 / (tol * tol), 1.0)
    return ReliableResult(X, iters, updates, status, np.sqrt(rho_true / bn2), np.sqrt(np.maximum(rho, 0) / bn2))
