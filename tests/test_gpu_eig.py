"""GPU parity of cola_eig_solve (Kronecker-eigen direct solve) against the oracle's direct solves."""
import numpy as np
import pytest

import workloads as wl
from oracle import direct, kron

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("dims,kind,sigma2", [((8, 12), "rbf", 0.1), ((5, 7), "wishart", 0.3),
                                               ((6, 5, 7), "wishart", 0.2), ((9,), "rbf", 0.05),
                                               ((16, 16, 16), "rbf", 0.01)])
def test_eig_solve_matches_cholesky(dims, kind, sigma2):
    """Odd and even mode sizes (the Jacobi ordering's idle slot), one to three modes."""
    from gpu_util import make_op, pack, unpack
    rng = np.random.default_rng(61)
    s = wl.random_system(rng, dims, nterms=1, diag=False, sigma2=sigma2, kind=kind)
    nrhs = 3
    B = rng.standard_normal((nrhs, s.n))
    op = make_op([s], prec="fp64")
    X = unpack(op.eig_solve(pack([B]), nrhs), [s], nrhs)[0]
    xref = direct.cholesky_solve(s.factors, B, s.sigma2)
    kappa = direct.condition_number(s.factors[0], s.sigma2)
    assert _rel(X, xref) <= max(1e-12, 50 * kappa * 2.2e-16), _rel(X, xref)
    assert np.all(kron.relres(s.factors, X, B, s.sigma2) <= 1e-12)
    # a second call reuses the decomposition
    X2 = unpack(op.eig_solve(pack([B]), nrhs), [s], nrhs)[0]
    assert np.array_equal(X, X2)
    op.close()


def test_eig_solve_several_systems():
    from gpu_util import make_op, pack, unpack
    rng = np.random.default_rng(62)
    systems = [wl.random_system(rng, d, nterms=1, diag=False, sigma2=0.1 + 0.1 * i)
               for i, d in enumerate([(4, 5), (3, 3, 3), (10,), (17, 6)])]
    nrhs = 2
    Bs = [rng.standard_normal((nrhs, s.n)) for s in systems]
    op = make_op(systems, prec="fp32")
    Xs = unpack(op.eig_solve(pack(Bs), nrhs), systems, nrhs)
    for s, B, X in zip(systems, Bs, Xs):
        assert _rel(X, direct.cholesky_solve(s.factors, B, s.sigma2)) <= 1e-11
    op.close()


@pytest.mark.parametrize("nterms,diag", [(2, False), (1, True)])
def test_eig_solve_rejects_other_structure(nterms, diag):
    from gpu_util import make_op, pack
    from paper_2309_03060_amd import ColaError
    rng = np.random.default_rng(63)
    s = wl.random_system(rng, (4, 6), nterms=nterms, diag=diag, sigma2=0.1)
    op = make_op([s], prec="fp64")
    with pytest.raises(ColaError) as e:
        op.eig_solve(pack([rng.standard_normal((1, s.n))]), 1)
    assert e.value.status == -6      # COLA_ERR_UNSUPPORTED
    op.close()


@pytest.mark.parametrize("cfg,tol", [("c2", 1e-9), ("c4", 1e-8)])
def test_eig_solve_full_size_certified(cfg, tol):
    """The 64^3 x 32 and 256^3 x 8 RBF operators solved directly; the oracle certifies the FP64 residual
    (bounded by about kappa * eps: kappa is 1.3e6 and 1.4e7)."""
    from gpu_util import make_op, pack, unpack
    w = wl.config2() if cfg == "c2" else wl.config4()
    s = w.systems[0]
    nrhs = w.B[0].shape[0]
    op = make_op([s], prec="fp32")
    X = unpack(op.eig_solve(pack(w.B), nrhs), [s], nrhs)[0]
    rr = kron.relres(s.factors, X, w.B[0], s.sigma2)
    assert np.all(rr <= tol), rr
    op.close()
