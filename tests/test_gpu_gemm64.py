"""The FP64 two-GEMM engine (two-mode operators with modes multiples of 256).

Every FP64 pass of such an operator runs on it: products, plain FP64 CG, and the FP64
residuals b - A x that certify mixed-precision solves (reliable updates and restarted
refinement).  Checked against the oracle's FP64 Kronecker product element by element (to
the rounding of a 2 n-term FP64 sum), against the general contraction passes with the engine
switched off, and end to end on solves certified by the oracle's residual.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import cg as ocg
from oracle import kron

pytestmark = pytest.mark.gpu


def _fp64_bound(s, X):
    """Elementwise bound on the rounding of the FP64 product: n_k-term sums of |factor| |x| per mode."""
    absf = [[np.abs(f) for f in row] for row in s.factors]
    dabs = None if s.diag is None else np.abs(s.diag)
    return kron.mvm(absf, np.abs(X), abs(s.sigma2), dabs)


@pytest.mark.parametrize("dims,nterms,diag,nrhs", [((256, 256), 1, True, 2), ((512, 256), 3, True, 3),
                                                   ((256, 768), 2, False, 1)])
def test_fp64_product_against_oracle(dims, nterms, diag, nrhs):
    import torch
    from gpu_util import make_op, pack, unpack
    rng = np.random.default_rng(sum(dims) + nterms)
    s = wl.random_system(rng, dims, nterms=nterms, diag=diag, sigma2=0.3)
    X = rng.standard_normal((nrhs, s.n))
    op = make_op([s], prec="bf16" if nterms > 1 else "fp32")
    op.profile_enable(True)
    Y = unpack(op.matvec(pack([X]), nrhs, prec="fp64"), [s], nrhs)[0]
    torch.cuda.synchronize()
    _, launches = op.profile_read("gemm_mode1_fp64")
    op.profile_enable(False)
    assert launches == 1
    op.set_engine("gemm64", False)
    Yg = unpack(op.matvec(pack([X]), nrhs, prec="fp64"), [s], nrhs)[0]
    op.close()
    ref = kron.mvm(s.factors, X, s.sigma2, s.diag)
    bound = _fp64_bound(s, X)
    k = nterms * dims[0] + dims[1] + 2      # terms in the longest FP64 sum chain (both modes, all terms)
    assert np.all(np.abs(Y - ref) <= k * 2.0 ** -53 * bound), np.max(np.abs(Y - ref) / bound)
    assert np.all(np.abs(Y - Yg) <= k * 2.0 ** -52 * bound)


def test_fp64_cg_on_engine_matches_oracle_and_general_path():
    """Plain FP64 CG (pack, G1, G2 with the CG epilogue) against the oracle's textbook CG: the same
    iteration count to within one, both solutions certified by the oracle's residual, and the
    general contraction path agreeing."""
    import torch
    from gpu_util import infos, make_op, pack, unpack
    rng = np.random.default_rng(64)
    s = wl.random_system(rng, (256, 512), nterms=2, diag=True, sigma2=0.05)
    nrhs = 2
    B = rng.standard_normal((nrhs, s.n))
    op = make_op([s], prec="bf16")
    op.profile_enable(True)
    X, info = op.solve(pack([B]), nrhs, prec="fp64", tol=1e-11, max_iters=2000)
    torch.cuda.synchronize()
    _, launches = op.profile_read("gemm_pack_fp64")
    op.profile_enable(False)
    rec = infos(info, nrhs)
    Xh = unpack(X, [s], nrhs)[0]
    op.set_engine("gemm64", False)
    X2, info2 = op.solve(pack([B]), nrhs, prec="fp64", tol=1e-11, max_iters=2000)
    rec2 = infos(info2, nrhs)
    X2h = unpack(X2, [s], nrhs)[0]
    op.close()
    assert launches >= 10
    res = ocg.cg(lambda V: kron.mvm(s.factors, V, s.sigma2, s.diag), B, tol=1e-11, max_iters=2000)
    rr = kron.relres(s.factors, Xh, B, s.sigma2, s.diag)
    rr2 = kron.relres(s.factors, X2h, B, s.sigma2, s.diag)
    for r in range(nrhs):
        assert rec[r]["status"] == 0 and rec2[r]["status"] == 0
        assert abs(rec[r]["iters"] - int(res.iters[r])) <= 1, (rec[r], res.iters[r])
        assert abs(rec[r]["iters"] - rec2[r]["iters"]) <= 1
        assert rr[r] <= 2e-11 and rr2[r] <= 2e-11, (rr, rr2)
        assert abs(rec[r]["relres_true"] - rr[r]) <= 1e-3 * rr[r] + 1e-16


@pytest.mark.parametrize("refine", ["reliable", "restart"])
def test_mixed_solve_residuals_on_engine(refine):
    """BF16 working precision on the BF16 GEMM engine, its FP64 residuals (EPI_RESID_CG with the
    per-RHS gate, or EPI_RESID of restarted refinement) on the FP64 engine: certified to 1e-10 by the
    oracle's residual, the reported true residual equal to the oracle's."""
    import torch
    from gpu_util import infos, make_op, pack, unpack
    rng = np.random.default_rng(65 if refine == "reliable" else 66)
    s = wl.random_system(rng, (512, 256), nterms=2, diag=True, sigma2=0.1)
    nrhs = 3
    B = rng.standard_normal((nrhs, s.n))
    op = make_op([s], prec="bf16")
    kw = dict(prec="bf16", tol=1e-10, max_iters=3000, check_every=32)
    if refine == "restart":
        kw.update(refine="restart", inner_tol=1e-2, max_sweeps=40)
    else:
        kw.update(inner_tol=0.1)
    op.profile_enable(True)
    X, info = op.solve(pack([B]), nrhs, **kw)
    torch.cuda.synchronize()
    _, launches = op.profile_read("gemm_mode1_fp64")
    op.profile_enable(False)
    rec = infos(info, nrhs)
    op.close()
    assert launches >= 2
    Xh = unpack(X, [s], nrhs)[0]
    rr = kron.relres(s.factors, Xh, B, s.sigma2, s.diag)
    for i, r in zip(rec, rr):
        assert i["status"] == 0 and r <= 1e-10, (rec, rr)
        assert abs(i["relres_true"] - r) <= 1e-3 * r, (i, r)


# One-term three-mode operators with every mode a multiple of 256: three FP64 GEMM passes, the
# last with the epilogue (the FP64 side of the 256^3 workload: plain FP64 CG and the residuals of
# its mixed-precision solves).
@pytest.mark.parametrize("dims,diag,nrhs", [((256, 256, 256), True, 2), ((512, 256, 256), False, 1)])
def test_fp64_three_mode_product_against_oracle(dims, diag, nrhs):
    import torch
    from gpu_util import make_op, pack, unpack
    rng = np.random.default_rng(sum(dims) + nrhs)
    s = wl.random_system(rng, dims, nterms=1, diag=diag, sigma2=0.3)
    X = rng.standard_normal((nrhs, s.n))
    op = make_op([s], prec="fp32")
    op.profile_enable(True)
    Y = unpack(op.matvec(pack([X]), nrhs, prec="fp64"), [s], nrhs)[0]
    torch.cuda.synchronize()
    _, launches = op.profile_read("gemm_mode3_fp64")
    op.profile_enable(False)
    assert launches == 1
    op.set_engine("gemm64", False)
    Yg = unpack(op.matvec(pack([X]), nrhs, prec="fp64"), [s], nrhs)[0]
    op.close()
    ref = kron.mvm(s.factors, X, s.sigma2, s.diag)
    bound = _fp64_bound(s, X)
    k = sum(dims) + 2
    assert np.all(np.abs(Y - ref) <= k * 2.0 ** -53 * bound), np.max(np.abs(Y - ref) / bound)
    assert np.all(np.abs(Y - Yg) <= k * 2.0 ** -52 * bound)


def test_fp64_three_mode_cg_and_mixed_residuals():
    """256^3 Wishart operator: plain FP64 CG on the engine (pack + three passes with the CG epilogue)
    against the general passes (iteration counts within one, both certified by the oracle's
    residual), and a BF16x3 solve whose FP64 reliable-update residuals run on the engine, certified
    to 1e-9 with its reported true residual equal to the oracle's."""
    import torch
    from gpu_util import infos, make_op, pack, unpack
    rng = np.random.default_rng(256)
    s = wl.random_system(rng, (256, 256, 256), nterms=1, diag=False, sigma2=0.1)
    nrhs = 2
    B = rng.standard_normal((nrhs, s.n))
    op = make_op([s], prec="bf16x3")
    op.profile_enable(True)
    X, info = op.solve(pack([B]), nrhs, prec="fp64", tol=1e-10, max_iters=500)
    torch.cuda.synchronize()
    _, launches = op.profile_read("gemm_pack_fp64")
    op.profile_enable(False)
    rec = infos(info, nrhs)
    Xh = unpack(X, [s], nrhs)[0]
    Xm, infom = op.solve(pack([B]), nrhs, prec="bf16x3", tol=1e-9, max_iters=2000, inner_tol=0.1)
    recm = infos(infom, nrhs)
    Xmh = unpack(Xm, [s], nrhs)[0]
    op.set_engine("gemm64", False)
    X2, info2 = op.solve(pack([B]), nrhs, prec="fp64", tol=1e-10, max_iters=500)
    rec2 = infos(info2, nrhs)
    op.close()
    assert launches >= 5
    rr = kron.relres(s.factors, Xh, B, s.sigma2)
    rr2 = kron.relres(s.factors, unpack(X2, [s], nrhs)[0], B, s.sigma2)
    rrm = kron.relres(s.factors, Xmh, B, s.sigma2)
    for r in range(nrhs):
        assert rec[r]["status"] == 0 and rec2[r]["status"] == 0 and recm[r]["status"] == 0
        assert abs(rec[r]["iters"] - rec2[r]["iters"]) <= 1, (rec, rec2)
        assert rr[r] <= 2e-10 and rr2[r] <= 2e-10, (rr, rr2)
        assert abs(rec[r]["relres_true"] - rr[r]) <= 1e-3 * rr[r]
        assert rrm[r] <= 1e-9 and abs(recm[r]["relres_true"] - rrm[r]) <= 1e-3 * rrm[r], (recm, rrm)
