"""Batched uneven systems (resident persistent kernel) against the oracle."""
import numpy as np
import pytest

import workloads as wl
from oracle import direct, grad, kron

pytestmark = pytest.mark.gpu


def _check_solutions(systems, Bs, Xs, infos, tol, fwd_factor=2.0):
    for s, B, X, i in zip(systems, Bs, Xs, infos):
        assert i["status"] == 0, i
        rr = kron.relres(s.factors, X, B, s.sigma2, s.diag)
        assert np.all(rr <= tol * (1 + 1e-9)), (rr, i)
        xref = direct.solve(s.factors, B, s.sigma2, s.diag)
        kappa = direct.condition_number(s.factors[0], s.sigma2) if s.diag is None else 1e3
        assert np.linalg.norm(X - xref) <= fwd_factor * kappa * tol * np.linalg.norm(xref) + 1e-300


def test_uneven_batch_reduced_all_systems():
    from gpu_util import infos, make_op, pack, unpack
    w = wl.config3(nsys=24, dmin=16, dmax=128, seed=31)
    op = make_op(w.systems, prec="fp32")
    X, info = op.solve(pack(w.B), 1, tol=1e-6, max_iters=5000)
    Xs = unpack(X, w.systems, 1)
    _check_solutions(w.systems, w.B, Xs, infos(info, len(w.systems)), 1e-6)
    op.close()


def test_uneven_batch_matches_single_system_path():
    """The resident batched kernel and the per-system streaming path agree."""
    from gpu_util import infos, make_op, pack, unpack
    w = wl.config3(nsys=5, dmin=9, dmax=70, seed=32)
    op = make_op(w.systems, prec="fp32")
    Xb, _ = op.solve(pack(w.B), 1, tol=1e-9, max_iters=5000)
    Xb = unpack(Xb, w.systems, 1)
    op.close()
    for s, B, xb in zip(w.systems, w.B, Xb):
        op1 = make_op([s], prec="fp32")            # one system: streaming path
        x1, i1 = op1.solve(pack([B]), 1, tol=1e-9, max_iters=5000)
        x1 = unpack(x1, [s], 1)[0]
        assert infos(i1, 1)[0]["status"] == 0
        xref = direct.kron_eig_solve(s.factors[0], B, s.sigma2)
        kappa = direct.condition_number(s.factors[0], s.sigma2)
        assert np.linalg.norm(xb - x1) <= 4 * kappa * 1e-9 * np.linalg.norm(xref)
        op1.close()


def test_uneven_batch_several_rhs_and_edge_cases():
    from gpu_util import infos, make_op, pack, unpack
    rng = np.random.default_rng(33)
    systems = [wl.random_system(rng, d, kind="rbf", sigma2=0.05, diag=(i % 2 == 1))
               for i, d in enumerate([(16, 16), (17, 33), (128, 128), (40, 100), (1, 64), (64, 1)])]
    nrhs = 3
    Bs = [rng.standard_normal((nrhs, s.n)) for s in systems]
    Bs[1][2] = 0.0                                   # zero right-hand side
    op = make_op(systems, prec="fp32")
    X, info = op.solve(pack(Bs), nrhs, tol=1e-7, max_iters=8000)
    Xs = unpack(X, systems, nrhs)
    inf = infos(info, len(systems) * nrhs)
    for k, (s, B, Xk) in enumerate(zip(systems, Bs, Xs)):
        for r in range(nrhs):
            i = inf[k * nrhs + r]
            assert i["status"] == 0, (k, r, i)
            if not B[r].any():
                assert i["iters"] == 0 and not Xk[r].any()
                continue
            assert kron.relres(s.factors, Xk[r:r + 1], B[r:r + 1], s.sigma2, s.diag)[0] <= 1e-7
    op.close()


@pytest.mark.slow
def test_uneven_batch_full_256_systems():
    """The full 256-system workload (dims U{16..128}) to 1e-5, every system certified by the oracle."""
    from gpu_util import infos, make_op, pack, unpack
    w = wl.config3()
    op = make_op(w.systems, prec="fp32")
    X, info = op.solve(pack(w.B), 1, tol=1e-5, max_iters=20000)
    Xs = unpack(X, w.systems, 1)
    _check_solutions(w.systems, w.B, Xs, infos(info, len(w.systems)), 1e-5)
    op.close()


def test_uneven_batch_gradients_against_oracle():
    """Adjoint gradients of L = sum_s w_s^T x_s over a batch: factors and sigma2 (1e-4 relative)."""
    from gpu_util import make_op, pack, unpack
    w = wl.config3(nsys=12, dmin=16, dmax=96, seed=34)
    op = make_op(w.systems, prec="fp32")
    kw = dict(tol=1e-10, max_iters=8000)
    X, _ = op.solve(pack(w.B), 1, **kw)
    Lam, dfac, _, ds2, _ = op.solve_backward(X, pack(w.W), 1, **kw)
    for k, s in enumerate(w.systems):
        Xr = direct.kron_eig_solve(s.factors[0], w.B[k], s.sigma2)
        Lr = direct.kron_eig_solve(s.factors[0], w.W[k], s.sigma2)
        g = grad.grad_kron(s.factors, Xr, Lr)
        for f in range(2):
            got = dfac[k][0][f].cpu().numpy()
            assert np.linalg.norm(got - g[0][0][f]) <= 1e-4 * np.linalg.norm(g[0][0][f]), (k, f)
        assert abs(float(ds2[k]) - g[2]) <= 1e-4 * abs(g[2]), k
    op.close()


def test_uneven_batch_gradients_two_rhs_fresh_op():
    """The resident solve sizes the shared workspace for one right-hand side; the adjoint backward of a
    fresh op with two right-hand sides must still stage its factor contractions for both (regression:
    the backward now sizes the workspace itself)."""
    from gpu_util import make_op, pack
    w = wl.config3(nsys=4, dmin=16, dmax=48, seed=35)
    rng = np.random.default_rng(36)
    nrhs = 2
    Bs = [rng.standard_normal((nrhs, s.n)) for s in w.systems]
    Ws = [rng.standard_normal((nrhs, s.n)) for s in w.systems]
    op = make_op(w.systems, prec="fp32")
    kw = dict(tol=1e-10, max_iters=8000)
    X, _ = op.solve(pack(Bs), nrhs, **kw)
    Lam, dfac, _, ds2, _ = op.solve_backward(X, pack(Ws), nrhs, **kw)
    for k, s in enumerate(w.systems):
        Xr = direct.kron_eig_solve(s.factors[0], Bs[k], s.sigma2)
        Lr = direct.kron_eig_solve(s.factors[0], Ws[k], s.sigma2)
        g = grad.grad_kron(s.factors, Xr, Lr)
        for f in range(2):
            got = dfac[k][0][f].cpu().numpy()
            assert np.linalg.norm(got - g[0][0][f]) <= 1e-4 * np.linalg.norm(g[0][0][f]), (k, f)
        assert abs(float(ds2[k]) - g[2]) <= 1e-4 * abs(g[2]), k
    op.close()
