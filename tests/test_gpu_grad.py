"""GPU parity of cola_cg_solve_backward and the autograd Function against the oracle gradients."""
import numpy as np
import pytest

import workloads as wl
from oracle import direct, grad

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


@pytest.mark.parametrize("dims,nterms,diag,prec", [((6, 9), 1, False, "fp64"), ((5, 4, 6), 2, True, "fp32"),
                                                   ((24, 20), 2, True, "bf16x3")])
def test_backward_matches_oracle_closed_forms(dims, nterms, diag, prec):
    from gpu_util import make_op, pack, unpack
    rng = np.random.default_rng(51)
    s = wl.random_system(rng, dims, nterms=nterms, diag=diag, sigma2=0.2)
    nrhs = 2
    B = rng.standard_normal((nrhs, s.n))
    W = rng.standard_normal((nrhs, s.n))
    Xref = direct.cholesky_solve(s.factors, B, s.sigma2, s.diag)
    Lref = direct.cholesky_solve(s.factors, W, s.sigma2, s.diag)
    gref = grad.grad_kron(s.factors, Xref, Lref, diag)
    op = make_op([s], prec="fp32" if prec == "fp64" else prec)
    kw = dict(tol=1e-11, max_iters=4000, prec=prec)
    X, _ = op.solve(pack([B]), nrhs, **kw)
    Lam, dfac, ddiag, ds2, info = op.solve_backward(X, pack([W]), nrhs, **kw)
    assert _rel(unpack(Lam, [s], nrhs)[0], Lref) <= 1e-8
    for j in range(nterms):
        for k in range(len(dims)):
            assert _rel(dfac[0][j][k].cpu().numpy(), gref[0][j][k]) <= 1e-6
    if diag:
        assert _rel(ddiag[0].cpu().numpy(), gref[1]) <= 1e-6
    assert abs(float(ds2[0]) - gref[2]) <= 1e-6 * abs(gref[2])
    op.close()


def test_backward_pinned_to_finite_differences_small():
    from gpu_util import make_op, pack
    rng = np.random.default_rng(52)
    s = wl.random_system(rng, (3, 4), nterms=1, diag=True, sigma2=0.3)
    B = rng.standard_normal((1, 12))
    W = rng.standard_normal((1, 12))
    op = make_op([s], prec="fp64")
    X, _ = op.solve(pack([B]), 1, tol=1e-13, max_iters=200, prec="fp64")
    _, dfac, ddiag, ds2, _ = op.solve_backward(X, pack([W]), 1, tol=1e-13, max_iters=200, prec="fp64")
    fd = grad.grad_fd(s.factors, s.sigma2, s.diag, B, W, ("factor", 0, 1, 2, 3))
    assert abs(dfac[0][0][1].cpu().numpy()[2, 3] - fd) <= 1e-6 * max(1.0, abs(fd))
    fd = grad.grad_fd(s.factors, s.sigma2, s.diag, B, W, ("sigma2",))
    assert abs(float(ds2[0]) - fd) <= 1e-6 * max(1.0, abs(fd))
    op.close()


def test_autograd_lengthscale_and_sigma2_uneven_batch():
    """Uneven-batch recipe (reduced): dL/dl through torch's RBF build, dL/dsigma2, dL/dB."""
    import torch
    from paper_2309_03060_amd import SystemSpec, kron_cg_solve
    w = wl.config3(nsys=4, dmin=6, dmax=20)
    dev = "cuda:0"
    specs, ells, pts = [], [], []
    for s in w.systems:
        facs = []
        for p, ell in zip(s.points, s.lengthscales):
            pt = torch.tensor(p, dtype=torch.float64, device=dev)
            lt = torch.tensor(ell, dtype=torch.float64, device=dev, requires_grad=True)
            ells.append(lt)
            d = pt[:, None] - pt[None, :]
            facs.append(torch.exp(-(d * d) / (2 * lt * lt)))
        s2 = torch.tensor(s.sigma2, dtype=torch.float64, device=dev, requires_grad=True)
        specs.append(SystemSpec(factors=[facs], sigma2=s2))
    B = torch.cat([torch.tensor(b.reshape(-1), device=dev) for b in w.B]).requires_grad_(True)
    Wt = torch.cat([torch.tensor(x.reshape(-1), device=dev) for x in w.W])
    X = kron_cg_solve(specs, B, 1, tol=1e-11, max_iters=4000, prec="fp32")
    loss = (X * Wt).sum()
    loss.backward()
    li = 0
    off = 0
    for si, s in enumerate(w.systems):
        Xr = direct.kron_eig_solve(s.factors[0], w.B[si], s.sigma2)
        Lr = direct.kron_eig_solve(s.factors[0], w.W[si], s.sigma2)
        g = grad.grad_kron(s.factors, Xr, Lr)
        for k in range(2):
            ref = grad.rbf_lengthscale_grad(g[0][0][k], s.factors[0][k], s.points[k], s.lengthscales[k])
            got = float(ells[li].grad)
            assert abs(got - ref) <= 1e-4 * abs(ref) + 1e-10, (si, k, got, ref)
            li += 1
        assert abs(float(specs[si].sigma2.grad) - g[2]) <= 1e-4 * abs(g[2])
        gb = B.grad[off:off + s.n].cpu().numpy()
        assert _rel(gb, Lr[0]) <= 1e-6
        off += s.n
