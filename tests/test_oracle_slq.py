"""Pins of the SLQ log-determinant oracle against facts fixed by the mathematics:

* the CG-Lanczos relation: the tridiagonal built from CG coefficients equals the
  tridiagonal of Lanczos with full reorthogonalisation on the same start vector;
* Gauss quadrature with a full Krylov space (m = n) is exact: it equals
  b^T log(A) b from the dense eigendecomposition;
* the Kronecker closed form of log det equals the dense log-determinant;
* the Hutchinson mean over many probes falls within its statistical error of the
  exact log det, and the probe estimate of d log det / d sigma2 of Tr(A^{-1});
* for one Kronecker factor the probe estimate of d log det / dK1 matches the
  dense derivative (A^{-1} restricted to the factor's Kronecker structure).
"""
import numpy as np

import workloads as wl
from oracle import kron, slq


def _spd(rng, n, shift=0.3):
    w = rng.standard_normal((n, n))
    return w @ w.T / n + shift * np.eye(n)


def _mvm(terms, sigma2, diag=None):
    return lambda V: kron.mvm(terms, V, sigma2, diag)


def test_cg_tridiagonal_equals_lanczos():
    rng = np.random.default_rng(1)
    A = _spd(rng, 40)
    apply_A = lambda V: V @ A.T
    b = rng.standard_normal(40)
    a, beta = slq.cg_coefficients(apply_A, b, 12)
    d, e = slq.tridiagonal_from_cg(a, beta)
    dl, el = slq.lanczos(apply_A, b, 12)
    assert len(d) == len(dl) == 12
    np.testing.assert_allclose(d, dl, rtol=1e-9, atol=0)
    np.testing.assert_allclose(e, el, rtol=1e-9, atol=0)          # both positive by construction


def test_full_krylov_quadrature_is_exact():
    rng = np.random.default_rng(2)
    n = 24
    A = _spd(rng, n, shift=0.5)
    b = rng.standard_normal(n)
    d, e = slq.lanczos(lambda V: V @ A.T, b, n)
    w, V = np.linalg.eigh(A)
    exact = float(b @ (V @ (np.log(w) * (V.T @ b))))
    got = float(b @ b) * slq.quadrature(d, e, np.log)
    assert abs(got - exact) <= 1e-9 * abs(exact)
    # a single CG iteration gives the one-node rule: log of the Rayleigh quotient
    a, beta = slq.cg_coefficients(lambda V: V @ A.T, b, 1)
    d1, e1 = slq.tridiagonal_from_cg(a, beta)
    assert abs(d1[0] - float(b @ A @ b) / float(b @ b)) <= 1e-12 * d1[0]


def test_kron_logdet_closed_form_matches_dense():
    rng = np.random.default_rng(3)
    facs = [_spd(rng, k, 0.2) for k in (5, 4, 3)]
    sign, ld = np.linalg.slogdet(kron.dense_operator([facs], 0.1))
    assert sign > 0
    assert abs(slq.kron_logdet(facs, 0.1) - ld) <= 1e-10 * abs(ld)
    Ainv = np.linalg.inv(kron.dense_operator([facs], 0.1))
    assert abs(slq.kron_trace_inverse(facs, 0.1) - np.trace(Ainv)) <= 1e-10 * np.trace(Ainv)


def test_slq_mean_within_statistical_error():
    rng = np.random.default_rng(4)
    facs = [_spd(rng, k, 0.3) for k in (6, 5, 4)]
    sigma2 = 0.5
    terms = [facs]
    Z = wl.rademacher_probes(rng, 1500, 120)
    est = slq.probe_logdets(_mvm(terms, sigma2), Z, 30)
    exact = slq.kron_logdet(facs, sigma2)
    err = abs(est.mean() - exact)
    assert err <= 4.0 * est.std(ddof=1) / np.sqrt(len(est)) + 1e-8 * abs(exact)
    # the same probes estimate Tr(A^{-1}) = d log det / d sigma2 through the solves
    Ainv = np.linalg.inv(kron.dense_operator(terms, sigma2))
    tr = np.einsum("ij,jk,ik->i", Z, Ainv, Z)
    assert abs(tr.mean() - slq.kron_trace_inverse(facs, sigma2)) <= 4.0 * tr.std(ddof=1) / np.sqrt(len(tr))


def test_probe_gradient_of_logdet_wrt_factor():
    """d log det A / dK1 = sum over the Kronecker structure of A^{-1}: the probe
    estimate mean_z (A^{-1} z)^T (dA/dK1[a, b]) z converges to it."""
    rng = np.random.default_rng(5)
    facs = [_spd(rng, 4, 0.3), _spd(rng, 5, 0.3)]
    sigma2 = 0.2
    A = kron.dense_operator([facs], sigma2)
    Ainv = np.linalg.inv(A)
    n1, n2 = 4, 5
    # exact: dlogdet/dK1[a, b] = Tr(A^{-1} (E_ab (x) K2)) = sum_{i, j} Ainv[(b, i), (a, j)] K2[i, j]
    Ai = Ainv.reshape(n1, n2, n1, n2)
    exact = np.einsum("bian,in->ab", Ai, facs[1])
    Z = wl.rademacher_probes(rng, 4000, n1 * n2)
    L = Z @ Ainv                                   # rows: A^{-1} z (A symmetric)
    # (A^{-1} z)^T (E_ab (x) K2) z = sum_{i, j} L[a, i] K2[i, j] Z[b, j]  per probe
    Lr, Zr = L.reshape(-1, n1, n2), Z.reshape(-1, n1, n2)
    per = np.einsum("pai,ij,pbj->pab", Lr, facs[1], Zr)
    mean, sd = per.mean(axis=0), per.std(axis=0, ddof=1) / np.sqrt(len(per))
    assert np.all(np.abs(mean - exact) <= 4.5 * sd + 1e-12)


def test_log_quadrature_equals_integral_form():
    """e1^T log(T) e1 = int_0^inf [1/(1+t) - e1^T (T + tI)^{-1} e1] dt for a positive definite tridiagonal
    T (the integral form of the matrix logarithm, which the device evaluates); checked here with an
    adaptive integrator against the eigendecomposition route, on Lanczos tridiagonals of a well and an
    ill conditioned operator."""
    import scipy.integrate
    rng = np.random.default_rng(6)
    for shift, m in ((0.5, 12), (1e-3, 40)):
        A = _spd(rng, 60, shift)
        d, e = slq.lanczos(lambda V: V @ A.T, rng.standard_normal(60), m)
        T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
        e1 = np.zeros(len(d))
        e1[0] = 1.0
        f = lambda t: 1.0 / (1.0 + t) - float(np.linalg.solve(T + t * np.eye(len(d)), e1)[0])
        # in u = log t the integrand is smooth and decays exponentially at both ends
        val, err = scipy.integrate.quad(lambda u: f(np.exp(u)) * np.exp(u), -60.0, 60.0, limit=400,
                                        epsabs=1e-13, epsrel=1e-12)
        ref = slq.quadrature(d, e, np.log)
        assert abs(val - ref) <= 1e-9 * max(1.0, abs(ref)), (shift, val, ref)
