"""GPU parity of the persistent fused CG (one-term K1 (x) K2 (x) K3 [+ diag], 64-wide modes, FP32
working precision): solutions certified by the oracle's FP64 residual and compared with the
separate-kernel path on the same inputs."""
import numpy as np
import pytest

import workloads as wl
from oracle import direct, kron

pytestmark = pytest.mark.gpu


def _wishart_system(seed, diag=True, sigma2=0.1):
    rng = np.random.default_rng(seed)
    facs = [wl.wishart_factor(rng, 64, shift=0.2) for _ in range(3)]
    d = rng.uniform(0.05, 0.5, size=64 ** 3) if diag else None
    return wl.System(factors=[facs], sigma2=sigma2, diag=d)


def _solve(s, B, nrhs, fused=True, **kw):
    from gpu_util import infos, make_op, pack, unpack
    op = make_op([s], prec="fp32")
    op.set_engine("fused_cg", fused)
    X, info = op.solve(pack([B]), nrhs, prec="fp32", **kw)
    out = unpack(X, [s], nrhs)[0], infos(info, nrhs)
    op.close()
    return out


def _certify(s, X, B, info, tol):
    rr = kron.relres(s.factors, X, B, s.sigma2, s.diag)
    bad = [(i, float(rr[i]), info[i]) for i in range(len(rr)) if not rr[i] <= tol]
    assert not bad, bad
    for i, r in zip(info, rr):
        assert i["status"] == 0, i
        assert abs(i["relres"] - r) <= 1e-3 * r + 1e-15     # the library's own FP64 residual
    return rr


@pytest.mark.parametrize("nrhs", [1, 5, 16, 17, 33])
def test_fused_reliable_with_diag(nrhs):
    """Every launch shape: 16 blocks per RHS (nrhs <= 16), 8 per RHS, and two launch batches (33)."""
    s = _wishart_system(7)
    B = np.random.default_rng(100 + nrhs).standard_normal((nrhs, s.n))
    X, info = _solve(s, B, nrhs, tol=1e-6, max_iters=2000, inner_tol=0.1)
    _certify(s, X, B, info, 1e-6)


def test_fused_rbf_matches_direct_solve():
    """The c2 operator (64^3 RBF, sigma2 0.01) to 1e-6: X against the oracle's Kronecker-eigen solve."""
    w = wl.config2(m=64, nrhs=3)
    s = w.systems[0]
    X, info = _solve(s, w.B[0], 3, tol=1e-6, max_iters=20000, inner_tol=0.1)
    _certify(s, X, w.B[0], info, 1e-6)
    xref = direct.kron_eig_solve(s.factors[0], w.B[0], s.sigma2)
    kappa = direct.condition_number(s.factors[0], s.sigma2)
    assert np.linalg.norm(X - xref) <= 2 * kappa * 1e-6 * np.linalg.norm(xref)


def test_fused_matches_separate_kernels_iteration_limit():
    """Stopped after 45 iterations (a chunk of 32 and a partial one): same status and iteration count as
    the separate-kernel path, and the same iterate up to FP32 rounding of the two reduction orders."""
    w = wl.config2(m=64, nrhs=4)
    s = w.systems[0]
    kw = dict(tol=1e-12, max_iters=45, inner_tol=0.1)
    Xf, inf_f = _solve(s, w.B[0], 4, fused=True, **kw)
    Xu, inf_u = _solve(s, w.B[0], 4, fused=False, **kw)
    for a, b in zip(inf_f, inf_u):
        assert a["status"] == b["status"] == 1, (a, b)
        assert a["iters"] == b["iters"] == 45, (a, b)
        assert abs(a["relres"] - b["relres"]) <= 1e-3 * b["relres"]
    assert np.linalg.norm(Xf - Xu) <= 1e-4 * np.linalg.norm(Xu)


def test_fused_restarted_refinement():
    """Restarted refinement runs plain FP32 CG inner solves (no reliable-update test in the kernel)."""
    s = _wishart_system(8, diag=False, sigma2=0.05)
    B = np.random.default_rng(9).standard_normal((3, s.n))
    X, info = _solve(s, B, 3, tol=1e-6, max_iters=2000, inner_tol=1e-4, max_sweeps=20, refine="restart")
    _certify(s, X, B, info, 1e-6)


def test_fused_zero_rhs_and_resume():
    """A zero right-hand side stops before the first iteration (x = 0); the others converge."""
    s = _wishart_system(10)
    B = np.random.default_rng(11).standard_normal((4, s.n))
    B[2] = 0.0
    X, info = _solve(s, B, 4, tol=1e-6, max_iters=2000, inner_tol=0.1)
    assert info[2]["status"] == 0 and info[2]["iters"] == 0
    assert np.all(X[2] == 0.0)
    keep = [0, 1, 3]
    _certify(s, X[keep], B[keep], [info[i] for i in keep], 1e-6)


def test_fused_engine_used_and_repeatable():
    """The fused launches are the ones timed (profile class cg_fused), and a repeated solve on the same
    op gives the same X bit for bit (fixed reduction orders)."""
    from gpu_util import make_op, pack, unpack
    s = _wishart_system(12)
    B = np.random.default_rng(13).standard_normal((6, s.n))
    op = make_op([s], prec="fp32")
    op.profile_enable(True)
    X1, _ = op.solve(pack([B]), 6, tol=1e-6, max_iters=2000, prec="fp32")
    ms, launches = op.profile_read("cg_fused")
    assert launches > 0
    assert op.profile_read("slab23")[1] == 0
    op.profile_enable(False)
    X2, _ = op.solve(pack([B]), 6, tol=1e-6, max_iters=2000, prec="fp32")
    assert np.array_equal(unpack(X1, [s], 6)[0], unpack(X2, [s], 6)[0])
    op.close()
