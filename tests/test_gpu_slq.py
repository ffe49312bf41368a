"""GPU parity of cola_slq_logdet (stochastic Lanczos quadrature of log det A) against the oracle:
per-probe estimates on the same probes, the closed-form Kronecker log det within the statistical
error of the probe mean, and the Hutchinson gradient of log det through the adjoint backward."""
import numpy as np
import pytest

import workloads as wl
from oracle import direct, grad, kron, slq

pytestmark = pytest.mark.gpu


def _mvm(s):
    return lambda V: kron.mvm(s.factors, V, s.sigma2, s.diag)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def test_slq_per_probe_matches_oracle_two_systems():
    """A three-mode RBF system and a two-term system with a diagonal in one op; CG run to 1e-10, so the
    quadrature uses each probe's whole Krylov history; one probe is zero (estimate 0, zero iterations)."""
    from gpu_util import infos, make_op, pack, unpack
    rng = np.random.default_rng(61)
    s1 = wl.random_system(rng, (10, 9, 8), nterms=1, sigma2=0.05, kind="rbf")
    s2 = wl.random_system(rng, (12, 11), nterms=2, diag=True, sigma2=0.1)
    nprobes = 6
    Z1 = wl.rademacher_probes(rng, nprobes, s1.n)
    Z2 = wl.rademacher_probes(rng, nprobes, s2.n)
    Z2[3] = 0.0
    op = make_op([s1, s2], prec="fp32")
    ld, est, X, info = op.logdet(pack([Z1, Z2]), nprobes, tol=1e-10, max_iters=400, want_solution=True)
    est = est.cpu().numpy().reshape(2, nprobes)
    ld = ld.cpu().numpy()
    inf = infos(info, 2 * nprobes)
    X1, X2 = unpack(X, [s1, s2], nprobes)
    for i, (s, Z, Xs) in enumerate(((s1, Z1, X1), (s2, Z2, X2))):
        ref = slq.probe_logdets(_mvm(s), Z, 400, tol=1e-10)
        assert np.all(np.abs(est[i] - ref) <= 1e-8 * np.abs(ref) + 1e-10), (i, est[i], ref)
        assert abs(ld[i] - ref.mean()) <= 1e-8 * abs(ref.mean())
        assert _rel(Xs, direct.cholesky_solve(s.factors, Z, s.sigma2, s.diag)) <= 1e-8
    assert est[1][3] == 0.0 and inf[nprobes + 3]["iters"] == 0
    assert all(r["status"] == 0 for r in inf)
    op.close()


@pytest.mark.parametrize("m", [1, 2, 7])
def test_slq_fixed_lanczos_steps(m):
    """max_iters = m caps the Krylov space: the same m-node rule as the oracle; m = 1 is the one-node rule
    ||z||^2 log(z^T A z / z^T z)."""
    from gpu_util import make_op, pack
    rng = np.random.default_rng(62 + m)
    s = wl.random_system(rng, (16, 12), nterms=1, diag=True, sigma2=0.2)
    Z = wl.rademacher_probes(rng, 5, s.n)
    op = make_op([s], prec="fp32")
    ld, est, _, _ = op.logdet(pack([Z]), 5, tol=1e-30, max_iters=m)
    est = est.cpu().numpy()
    ref = slq.probe_logdets(_mvm(s), Z, m)
    assert np.all(np.abs(est - ref) <= 1e-9 * np.abs(ref)), (est, ref)
    if m == 1:
        AZ = _mvm(s)(Z)
        one = np.einsum("ij,ij->i", Z, Z) * np.log(np.einsum("ij,ij->i", Z, AZ) / np.einsum("ij,ij->i", Z, Z))
        assert np.all(np.abs(est - one) <= 1e-10 * np.abs(one))
    op.close()


def test_slq_full_size_against_closed_form():
    """64^3 RBF factors of the benchmark workload with sigma2 = 0.1, 32 probes: the mean lies within its
    statistical error of the closed-form Kronecker log det; two probes match the oracle probe by probe."""
    from gpu_util import make_op, pack
    w = wl.config2()
    base = w.systems[0]
    s = wl.System(factors=base.factors, sigma2=0.1)
    rng = np.random.default_rng(63)
    nprobes = 32
    Z = wl.rademacher_probes(rng, nprobes, s.n)
    op = make_op([s], prec="fp32")
    ld, est, _, info = op.logdet(pack([Z]), nprobes, tol=1e-9, max_iters=300)
    est = est.cpu().numpy()
    exact = slq.kron_logdet(s.factors[0], s.sigma2)
    sd = est.std(ddof=1) / np.sqrt(nprobes)
    assert abs(float(ld[0]) - exact) <= 5.0 * sd, (float(ld[0]), exact, sd)
    ref = slq.probe_logdets(_mvm(s), Z[:2], 300, tol=1e-9)
    assert np.all(np.abs(est[:2] - ref) <= 1e-7 * np.abs(ref)), (est[:2], ref)
    op.close()


def test_logdet_gradient_through_backward():
    """d log det / d(factors, diagonal, sigma2) as the probe mean of (A^{-1} z)^T (dA/dtheta) z: equal to
    the oracle's closed-form contractions with X = Z, Lambda = A^{-1} Z on the same probes, and its sigma2
    component within the statistical error of Tr(A^{-1})."""
    from gpu_util import make_op, pack
    rng = np.random.default_rng(64)
    s = wl.random_system(rng, (6, 5, 4), nterms=1, diag=True, sigma2=0.3)
    nprobes = 256
    Z = wl.rademacher_probes(rng, nprobes, s.n)
    op = make_op([s], prec="fp32")
    dfac, ddiag, ds2, _ = op.logdet_grad(pack([Z]), nprobes, tol=1e-12, max_iters=2000)
    Lam = direct.cholesky_solve(s.factors, Z, s.sigma2, s.diag)
    gref = grad.grad_kron(s.factors, Z, Lam, True)
    for k in range(3):
        assert _rel(dfac[0][0][k].cpu().numpy(), -gref[0][0][k] / nprobes) <= 1e-8
    assert _rel(ddiag[0].cpu().numpy(), -gref[1] / nprobes) <= 1e-8
    assert abs(float(ds2[0]) + gref[2] / nprobes) <= 1e-8 * abs(gref[2] / nprobes)
    A = kron.dense_operator(s.factors, s.sigma2, s.diag)
    per = np.einsum("ij,ij->i", Z, Lam)
    assert abs(float(ds2[0]) - np.trace(np.linalg.inv(A))) <= 5.0 * per.std(ddof=1) / np.sqrt(nprobes)
    op.close()
