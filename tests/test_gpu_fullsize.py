"""Parity at the full workload sizes, with the tile shapes the autotuner picks.

Products are checked on sampled entries against the oracle's entry-wise
definition of (A x)[i]; solves are certified by the oracle's FP64 true
residual ||b - A x|| / ||b|| (which holds at any size); the sum-of-Kronecker
gradients are compared with the oracle's closed forms evaluated at the
solution and adjoint the GPU returned (both certified by their residuals).
"""
import numpy as np
import pytest

import workloads as wl
from oracle import grad, kron

pytestmark = pytest.mark.gpu


def _sampled_check(op, s, X, nrhs, prec, tol, rows, seed, k=5):
    import torch
    from gpu_util import pack, unpack
    dt = torch.float64 if prec == "fp64" else torch.float32
    Y = unpack(op.matvec(pack([X], dt), nrhs, prec=prec), [s], nrhs)[0]
    absf = [[np.abs(f) for f in row] for row in s.factors]
    absd = None if s.diag is None else np.abs(s.diag)
    rng = np.random.default_rng(seed)
    for r in rows:
        for idx in list(rng.integers(0, s.n, size=k)) + [0, s.n - 1]:
            ref = kron.mvm_entry(s.factors, X[r], int(idx), s.sigma2, s.diag)
            scale = kron.mvm_entry(absf, np.abs(X[r]), int(idx), s.sigma2, absd)
            assert abs(Y[r, idx] - ref) <= tol * scale, (prec, r, int(idx), Y[r, idx], ref)


def _certify(s, X, B, info, tol):
    rr = kron.relres(s.factors, X, B, s.sigma2, s.diag)
    bad = [(i, float(rr[i]), info[i]) for i in range(len(rr)) if not rr[i] <= tol]
    assert not bad, bad
    for i, r in zip(info, rr):
        assert i["status"] == 0, i
        assert abs(i["relres"] - r) <= 1e-3 * r + 1e-15     # the library's own FP64 residual
    return rr


@pytest.mark.parametrize("check_every", [128, 32])
def test_c2_full_solve_bench_configuration(check_every):
    """64^3 RBF operator, 32 RHS, FP32 CG with FP64 reliable updates to 1e-5 (the timed workload): 128
    fused CG iterations per launch and host check as the benchmark runs it, and 32."""
    from gpu_util import infos, make_op, pack, unpack
    w = wl.config2()
    s = w.systems[0]
    op = make_op([s], prec="fp32")
    op.autotune(32)
    X, info = op.solve(pack(w.B), 32, tol=1e-5, max_iters=20000, prec="fp32", inner_tol=0.1,
                       check_every=check_every)
    _certify(s, unpack(X, [s], 32)[0], w.B[0], infos(info, 32), 1e-5)
    op.close()


# FP32 accumulation over three length-256 contractions: the worst-case bound is about 3 * 256 * 2^-24
# of the absolute-value product (4.6e-5); observed errors are far smaller, 1e-5 still catches any
# wrong operand or dropped term (those give O(1) errors) and any BF16-only rounding (~4e-3).
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 1e-5), ("bf16x3", 1e-5)])
def test_c4_full_matvec_sampled(prec, tol):
    """256^3 RBF operator with 8 RHS: sampled product entries in every precision."""
    from gpu_util import make_op
    w = wl.config4()
    s = w.systems[0]
    op = make_op([s], prec="fp32" if prec == "fp64" else prec)
    op.autotune(8)
    _sampled_check(op, s, w.B[0], 8, prec, tol, rows=(0, 7), seed=41)
    op.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_c4_full_solve_certified(prec):
    """256^3 x 8 RHS mixed-precision solve, stopped at 1e-3 to keep the test short; the oracle
    certifies the returned X by its FP64 residual and checks the library's reported residual."""
    from gpu_util import infos, make_op, pack, unpack
    w = wl.config4()
    s = w.systems[0]
    op = make_op([s], prec=prec)
    op.autotune(8)
    X, info = op.solve(pack(w.B), 8, tol=1e-3, max_iters=20000, prec=prec, inner_tol=0.1, check_every=32)
    _certify(s, unpack(X, [s], 8)[0], w.B[0], infos(info, 8), 1e-3)
    op.close()


def test_c5_full_matvec_sampled():
    """Sum of four 1024^2 Kronecker terms plus diagonal, 16 RHS: sampled entries, FP64 and BF16."""
    from gpu_util import make_op
    w = wl.config5()
    s = w.systems[0]
    op = make_op([s], prec="bf16")
    _sampled_check(op, s, w.B[0], 16, "fp64", 1e-13, rows=(0, 15), seed=51)
    # BF16 operands: unit roundoff 2^-8 on each of the two factor products and on x
    _sampled_check(op, s, w.B[0], 16, "bf16", 2e-2, rows=(0, 15), seed=52)
    op.close()


def test_c5_full_solve_and_backward():
    """BF16 CG with FP64 reliable updates to 1e-6, then the adjoint backward: Lambda certified by
    its residual, factor / diagonal gradients against the oracle's closed forms at (X, Lambda)."""
    from gpu_util import infos, make_op, pack, unpack
    w = wl.config5()
    s = w.systems[0]
    nrhs = 16
    op = make_op([s], prec="bf16")
    op.autotune(nrhs)
    kw = dict(tol=1e-6, max_iters=2000, prec="bf16", inner_tol=0.1, check_every=32)
    X, info = op.solve(pack(w.B), nrhs, **kw)
    Xh = unpack(X, [s], nrhs)[0]
    _certify(s, Xh, w.B[0], infos(info, nrhs), 1e-6)
    Lam, dfac, ddiag, ds2, info2 = op.solve_backward(X, pack(w.W), nrhs, **kw)
    Lh = unpack(Lam, [s], nrhs)[0]
    _certify(s, Lh, w.W[0], infos(info2, nrhs), 1e-6)
    gref = grad.grad_kron(s.factors, Xh, Lh, True)
    for j in range(len(s.factors)):
        for k in range(2):
            got = dfac[0][j][k].cpu().numpy()
            assert np.linalg.norm(got - gref[0][j][k]) <= 1e-10 * np.linalg.norm(gref[0][j][k]), (j, k)
    assert np.linalg.norm(ddiag[0].cpu().numpy() - gref[1]) <= 1e-10 * np.linalg.norm(gref[1])
    op.close()
