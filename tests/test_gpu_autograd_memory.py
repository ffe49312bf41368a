"""Backward-pass memory and runtime of the adjoint rules (App. B.2, and App. B's figure comparing them
with unrolled autodiff): the library's backward holds a fixed set of buffers whatever the number of CG
steps, while autograd through an unrolled plain-torch CG stores every step.  The gradients of the two
agree once CG has converged, and the adjoint gradients match the oracle's closed forms."""
import numpy as np
import pytest

import bench
import workloads as wl
from oracle import direct, grad

pytestmark = pytest.mark.gpu

ELL, S2 = 0.15, 0.05


def _pts(m):
    return wl.config2(m=m, nrhs=1).systems[0].points


def test_adjoint_memory_flat_in_steps_unrolled_grows():
    pts = _pts(32)
    a = bench.autograd_solve_pair(pts, ELL, S2, 2, iters=32)
    b = bench.autograd_solve_pair(pts, ELL, S2, 2, iters=256)
    print("32 steps:", a, "\n256 steps:", b, flush=True)
    assert a["adjoint"]["iters"] == 32 and b["adjoint"]["iters"] == 256
    assert a["unrolled"]["iters"] == 32 and b["unrolled"]["iters"] == 256
    # the operator's buffers do not depend on the step count; torch holds the same tensors
    assert b["adjoint"]["library_peak_bytes"] == a["adjoint"]["library_peak_bytes"]
    assert b["adjoint"]["torch_peak_bytes"] <= 1.05 * a["adjoint"]["torch_peak_bytes"] + 2 ** 20
    # unrolled autodiff keeps every step: 8x the steps, at least 4x the memory (one vector of the
    # 32^3 operator is 256 KiB, so 256 steps store hundreds of MiB)
    assert b["unrolled"]["peak_bytes"] >= 4 * a["unrolled"]["peak_bytes"]
    assert b["unrolled"]["peak_bytes"] >= 4 * b["adjoint"]["peak_bytes"]


def test_adjoint_and_unrolled_gradients_agree_and_match_oracle():
    """Solved to 1e-11 on a 24^3 RBF operator with s2 = 1 (condition number about 760), two right-hand
    sides: dL/dl, dL/ds2 and dL/dB of the two paths agree to 1e-6, and the adjoint's match the oracle
    (Kronecker-eigen solves for X and Lambda, closed-form factor contractions, the RBF chain rule) to
    1e-6.  At s2 = 0.05 (condition number in the thousands) the unrolled gradient is not usable: reverse
    mode through a few hundred FP64 CG steps cancels adjoints of growing size, while central differences
    of the same k-step program agree with the oracle; that case is measured, not asserted."""
    m, nrhs, seed, s2 = 24, 2, 11, 1.0
    pts = _pts(m)
    r = bench.autograd_solve_pair(pts, ELL, s2, nrhs, tol=1e-11, seed=seed)
    print(r, flush=True)
    adj, unr = r["adjoint"], r["unrolled"]
    for key in ("grad_ell", "grad_sigma2"):
        assert abs(adj[key] - unr[key]) <= 1e-6 * abs(unr[key]), key
    assert unr["grad_B_rel_diff"] <= 1e-6
    # oracle: the same B and W (rows of N(0, 1) from default_rng(seed), B first)
    rng = np.random.default_rng(seed)
    n = m ** 3
    B = rng.standard_normal((nrhs, n))
    W = rng.standard_normal((nrhs, n))
    facs = [wl.rbf_kernel(p, ELL) for p in pts]
    X = direct.kron_eig_solve(facs, B, s2)
    Lam = direct.kron_eig_solve(facs, W, s2)
    dfac, _, ds2 = grad.grad_kron([facs], X, Lam)
    dell = sum(grad.rbf_lengthscale_grad(dfac[0][k], facs[k], pts[k], ELL) for k in range(3))
    assert abs(adj["grad_ell"] - dell) <= 1e-6 * abs(dell)
    assert abs(adj["grad_sigma2"] - ds2) <= 1e-6 * abs(ds2)


def test_logdet_adjoint_memory_flat_and_sigma2_gradient_matches_unrolled():
    """Log det by SLQ with exactly k Lanczos steps per probe: the adjoint path's memory does not depend
    on k; unrolled autodiff through CG, the tridiagonal and its eigendecomposition grows with k.  At any
    k both paths compute the same estimate, and the same d/ds2: the Lanczos tridiagonal of A + s2 I is
    T_k + s2 I, so d/ds2 of ||z||^2 e1^T log(T_k + s2 I) e1 is ||z||^2 e1^T (T_k + s2 I)^{-1} e1 = z^T x_k
    (x_k: k steps of CG on A x = z), which is what the adjoint backward with X = G = Z returns."""
    pts = _pts(16)
    a = bench.autograd_logdet_pair(pts, ELL, S2, 4, 16)
    b = bench.autograd_logdet_pair(pts, ELL, S2, 4, 128)
    print("16 steps:", a, "\n128 steps:", b, flush=True)
    # the adjoint path holds the n-sized workspace of a solve plus the CG coefficient history of the
    # quadrature (16 bytes per probe and step, independent of n)
    grow = b["adjoint"]["library_peak_bytes"] - a["adjoint"]["library_peak_bytes"]
    assert 0 <= grow <= 16 * 4 * (128 - 16)
    assert b["unrolled"]["peak_bytes"] >= 3 * a["unrolled"]["peak_bytes"]
    for r in (a, b):
        assert abs(r["adjoint"]["logdet"] - r["unrolled"]["logdet"]) <= 1e-8 * abs(r["unrolled"]["logdet"])
    g_adj, g_unr = a["adjoint"]["grad_sigma2"], a["unrolled"]["grad_sigma2"]
    assert np.isfinite(g_unr) and abs(g_adj - g_unr) <= 1e-6 * abs(g_unr)
