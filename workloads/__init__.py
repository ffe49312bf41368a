"""Seeded synthetic inputs for the sum-of-Kronecker-plus-diagonal CG workloads.

This module only draws random numbers and builds the operator's *data*
(kernel-matrix factors, diagonals, right-hand sides, loss weights) in
float64 with numpy.  It holds none of the method's arithmetic (no MVM, no
CG, no gradient) and is the one piece of code shared by the CPU oracle and
the GPU path: both consume the arrays produced here.

Operator family (CoLA, Sec. 3.2 "compositional linear operators"):

    A = sum_j (K_j1 (x) K_j2 [(x) K_j3]) + diag(d) + sigma2 * I

Factors are either RBF kernel matrices on points in [0, 1]
(the multi-task GP operator of Fig. 1(a) and App. D.2 uses an RBF data
kernel) or Wishart-type SPD matrices W W^T / m + 0.1 I.

RBF reading: k(x, x') = exp(-(x - x')^2 / (2 l^2)) with unit amplitude
(the paper names the kernel but not its parametrisation).  Points are drawn
i.i.d. U[0, 1] and sorted (sorting permutes nothing in the spectrum).

Every generator takes an explicit seed and draws in a documented order, so
the same call returns bit-identical arrays on any machine with numpy's
PCG64.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


def rbf_kernel(points: np.ndarray, lengthscale: float) -> np.ndarray:
    """Dense RBF kernel matrix exp(-(x_i - x_j)^2 / (2 l^2)) in float64."""
    p = np.asarray(points, dtype=np.float64)
    diff = p[:, None] - p[None, :]
    return np.exp(-(diff * diff) / (2.0 * float(lengthscale) ** 2))


def wishart_factor(rng: np.random.Generator, m: int, shift: float = 0.1) -> np.ndarray:
    """SPD factor W W^T / m + shift * I with W ~ N(0, 1)^{m x m}."""
    w = rng.standard_normal((m, m))
    k = (w @ w.T) / m
    k = 0.5 * (k + k.T)
    k[np.diag_indices(m)] += shift
    return k


@dataclass
class System:
    """One SPD system A = sum_j kron(factors[j]) + diag(d) + sigma2 I.

    factors[j][k] is the k-th Kronecker factor of term j (row-major
    n_k x n_k float64); ``points`` / ``lengthscales`` are kept for RBF
    factors so lengthscale gradients can be formed by the chain rule.
    """
    factors: List[List[np.ndarray]]
    sigma2: float
    diag: Optional[np.ndarray] = None
    points: Optional[List[np.ndarray]] = None        # per factor of term 0 (RBF only)
    lengthscales: Optional[List[float]] = None       # per factor of term 0 (RBF only)

    @property
    def dims(self):
        return tuple(int(f.shape[0]) for f in self.factors[0])

    @property
    def n(self) -> int:
        return int(np.prod(self.dims))

    @property
    def nterms(self) -> int:
        return len(self.factors)

    @property
    def nfactors(self) -> int:
        return len(self.factors[0])


@dataclass
class Workload:
    """A batch of systems and right-hand sides.

    B[s] has shape (nrhs, n_s): each row is one right-hand side (contiguous,
    i.e. column-major n_s x nrhs).  W[s] (same shape) are loss weights for
    the loss L = sum_s sum_r w_sr^T x_sr used by the gradient workloads.
    """
    name: str
    systems: List[System]
    B: List[np.ndarray]
    W: List[np.ndarray] = field(default_factory=list)
    tol: float = 1e-6
    description: str = ""


def _rbf_system(rng, dims, lengthscale, sigma2):
    pts = [np.sort(rng.uniform(0.0, 1.0, size=m)) for m in dims]
    facs = [rbf_kernel(p, lengthscale) for p in pts]
    return System(factors=[facs], sigma2=float(sigma2), points=pts,
                  lengthscales=[float(lengthscale)] * len(dims))


def config1(m: int = 64, seed: int = 1) -> Workload:
    """K1 (x) K2 + 0.1 I, RBF l = 0.2 on m uniform points each, 1 RHS, FP64, tol 1e-10.

    Draw order: points of factor 1, points of factor 2, b.
    """
    rng = np.random.default_rng(seed)
    sys_ = _rbf_system(rng, (m, m), 0.2, 0.1)
    b = rng.standard_normal((1, sys_.n))
    return Workload("c1_kron2_fp64", [sys_], [b], tol=1e-10,
                    description=f"K1(x)K2+0.1I RBF l=0.2, {m}x{m}, 1 RHS")


def config2(m: int = 64, nrhs: int = 32, seed: int = 2) -> Workload:
    """K1 (x) K2 (x) K3 + 0.01 I, RBF l = 0.15, m points each, nrhs RHS, tol 1e-5.

    Draw order: points of factors 1, 2, 3, then B row by row.
    """
    rng = np.random.default_rng(seed)
    sys_ = _rbf_system(rng, (m, m, m), 0.15, 0.01)
    b = rng.standard_normal((nrhs, sys_.n))
    return Workload("c2_kron3_fp32", [sys_], [b], tol=1e-5,
                    description=f"K1(x)K2(x)K3+0.01I RBF l=0.15, {m}^3, {nrhs} RHS")


def config3(nsys: int = 256, dmin: int = 16, dmax: int = 128, seed: int = 3) -> Workload:
    """nsys independent K1 (x) K2 + sigma2 I systems of uneven size, 1 RHS each.

    Per system, in this order: d1, d2 ~ U{dmin..dmax}; l1, l2 ~ U[0.1, 0.5];
    sigma2 ~ U[0.01, 0.1]; points of factor 1; points of factor 2;
    b ~ N(0, 1)^n; w ~ N(0, 1)^n.  Each factor has its own lengthscale.
    """
    rng = np.random.default_rng(seed)
    systems, Bs, Ws = [], [], []
    for _ in range(nsys):
        d1, d2 = (int(v) for v in rng.integers(dmin, dmax + 1, size=2))
        l1, l2 = (float(v) for v in rng.uniform(0.1, 0.5, size=2))
        s2 = float(rng.uniform(0.01, 0.1))
        p1 = np.sort(rng.uniform(0.0, 1.0, size=d1))
        p2 = np.sort(rng.uniform(0.0, 1.0, size=d2))
        sys_ = System(factors=[[rbf_kernel(p1, l1), rbf_kernel(p2, l2)]], sigma2=s2,
                      points=[p1, p2], lengthscales=[l1, l2])
        systems.append(sys_)
        Bs.append(rng.standard_normal((1, sys_.n)))
        Ws.append(rng.standard_normal((1, sys_.n)))
    return Workload("c3_uneven_batch", systems, Bs, Ws, tol=1e-5,
                    description=f"{nsys} uneven K1(x)K2+s2 I systems, dims U{{{dmin}..{dmax}}}")


def config4(m: int = 256, nrhs: int = 8, seed: int = 4) -> Workload:
    """K1 (x) K2 (x) K3 + 0.05 I, RBF l = 0.15, m points each, nrhs RHS, tol 1e-6.

    Draw order as config2.
    """
    rng = np.random.default_rng(seed)
    sys_ = _rbf_system(rng, (m, m, m), 0.15, 0.05)
    b = rng.standard_normal((nrhs, sys_.n))
    return Workload("c4_kron3_mixed", [sys_], [b], tol=1e-6,
                    description=f"K1(x)K2(x)K3+0.05I RBF l=0.15, {m}^3, {nrhs} RHS")


def config5(m: int = 1024, nterms: int = 4, nrhs: int = 16, seed: int = 5) -> Workload:
    """sum_{j<nterms} U_j (x) V_j + diag(d), Wishart factors, d ~ U[0.1, 1], tol 1e-6.

    Draw order: for each term j: U_j's W, then V_j's W; then d; then B; then
    the loss weights W_loss.
    """
    rng = np.random.default_rng(seed)
    facs = []
    for _ in range(nterms):
        u = wishart_factor(rng, m)
        v = wishart_factor(rng, m)
        facs.append([u, v])
    n = m * m
    d = rng.uniform(0.1, 1.0, size=n)
    b = rng.standard_normal((nrhs, n))
    w = rng.standard_normal((nrhs, n))
    sys_ = System(factors=facs, sigma2=0.0, diag=d)
    return Workload("c5_sumkron_diag", [sys_], [b], [w], tol=1e-6,
                    description=f"sum_{nterms} U(x)V + diag(d), {m}^2, {nrhs} RHS")


def rademacher_probes(rng: np.random.Generator, count: int, n: int) -> np.ndarray:
    """count probe vectors of length n with independent +-1 entries (E[z z^T] = I)."""
    return np.where(rng.random((count, n)) < 0.5, -1.0, 1.0)


def random_system(rng: np.random.Generator, dims, nterms: int = 1, diag: bool = False,
                  sigma2: float = 0.1, kind: str = "wishart") -> System:
    """Small generic SPD system for parity sweeps (tiles, ragged tails, edge cases).

    kind = "wishart": each factor W W^T / m + 0.1 I;  kind = "rbf": RBF on U[0,1]
    points with lengthscale U[0.1, 0.5].  Draw order: factors term by term,
    factor by factor; then d ~ U[0.1, 1] if requested.
    """
    facs, pts, ls = [], [], []
    for _ in range(nterms):
        row = []
        for m in dims:
            if kind == "rbf":
                p = np.sort(rng.uniform(0.0, 1.0, size=m))
                ell = float(rng.uniform(0.1, 0.5))
                row.append(rbf_kernel(p, ell))
                pts.append(p)
                ls.append(ell)
            else:
                row.append(wishart_factor(rng, m))
        facs.append(row)
    d = rng.uniform(0.1, 1.0, size=int(np.prod(dims))) if diag else None
    return System(factors=facs, sigma2=float(sigma2), diag=d,
                  points=pts[:len(dims)] if kind == "rbf" else None,
                  lengthscales=ls[:len(dims)] if kind == "rbf" else None)


def random_rhs(rng: np.random.Generator, n: int, nrhs: int) -> np.ndarray:
    """Right-hand sides ~ N(0, 1), shape (nrhs, n)."""
    return rng.standard_normal((nrhs, n))


CONFIGS = {
    "c1": config1,
    "c2": config2,
    "c3": config3,
    "c4": config4,
    "c5": config5,
}
