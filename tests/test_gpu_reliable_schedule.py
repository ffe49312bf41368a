"""The library's mixed-precision schedules against the oracle's (oracle.cg.reliable, oracle.cg.refine).

Both sides follow one reading of the paper's low precision by algorithmic modification (Sec. 3.4,
App. C.3): a single FP32 CG whose residual is replaced by the FP64 true residual b - A x once it has
fallen by delta = inner_tol below the last replaced one, at the end of the chunk of check_every
iterations in which that happened (the resident batched kernel ends its chunk at the request, so its
chunks are of one iteration).  The two differ only in the FP32 summation order of the products, so
on well-conditioned systems the iteration counts agree to a few, the number of replacements to one
and the status exactly, and both solutions are certified by the FP64 residual and agree within the
forward-error bound.  Each case checks, from the profile classes, that the engine named ran.
Restarted refinement (refine="restart") is compared the same way with oracle.cg.refine: each sweep
an FP32 CG from zero on r / ||r|| to inner_tol, then x += ||r|| d in FP64; the same status and
number of sweeps, inner iterations summed over the sweeps within a few.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import cg as ocg
from oracle import kron, lowprec

pytestmark = pytest.mark.gpu


def _low(s):
    """The FP32 operator: factors, sigma^2 and d rounded to FP32 (the product rounded by the oracle)."""
    f32 = [[lowprec.to_fp32(f) for f in row] for row in s.factors]
    d32 = None if s.diag is None else lowprec.to_fp32(s.diag)
    s2 = float(np.float32(s.sigma2))
    return lambda V: kron.mvm(f32, V, s2, d32)


def _oracle(s, B, tol, delta, every, max_iters):
    A64 = lambda V: kron.mvm(s.factors, V, s.sigma2, s.diag)
    return ocg.reliable(A64, _low(s), B, tol=tol, delta=delta, max_iters=max_iters, check_every=every)


def _cond(s):
    if s.diag is None and len(s.factors) == 1:
        ev = [np.linalg.eigvalsh(f) for f in s.factors[0]]
        hi = np.prod([e.max() for e in ev]) + s.sigma2
        lo = np.prod([e.min() for e in ev]) + s.sigma2
        return float(hi / lo)
    if s.n <= 4096:
        return float(np.linalg.cond(kron.dense_operator(s.factors, s.sigma2, s.diag)))
    # a bound (Weyl): the Kronecker terms are PSD, each at most the product of its factors' largest
    # eigenvalues
    top = sum(np.prod([np.linalg.eigvalsh(f).max() for f in row]) for row in s.factors)
    dmin = 0.0 if s.diag is None else float(s.diag.min())
    dmax = 0.0 if s.diag is None else float(s.diag.max())
    return float((top + s.sigma2 + dmax) / (s.sigma2 + dmin))


def _compare(s, B, X, rec, ref, tol, iter_band):
    rr = kron.relres(s.factors, X, B, s.sigma2, s.diag)
    kappa = _cond(s)
    for i in range(B.shape[0]):
        assert rec[i]["status"] == 0 and ref.status[i] == "ok", (rec[i], ref.status[i])
        assert abs(rec[i]["iters"] - int(ref.iters[i])) <= iter_band, (i, rec[i], ref.iters)
        assert abs(rec[i]["sweeps"] - int(ref.updates[i])) <= 1, (i, rec[i], ref.updates)
        assert rr[i] <= tol and ref.relres_true[i] <= tol, (rr, ref.relres_true)
        assert abs(rec[i]["relres_true"] - rr[i]) <= 1e-3 * rr[i], (rec[i], rr[i])
        xn = np.linalg.norm(ref.X[i])
        assert np.linalg.norm(X[i] - ref.X[i]) <= 4.0 * kappa * tol * xn, (i, kappa)


def _solve(op, s, B, **kw):
    import torch
    from gpu_util import infos, pack, unpack
    nrhs = B.shape[0]
    X, info = op.solve(pack([B]), nrhs, prec="fp32", **kw)
    torch.cuda.synchronize()
    return unpack(X, [s], nrhs)[0], infos(info, nrhs)


def _launches(op, s, B, cls, **kw):
    """Launches of the profile classes cls in one more solve with profiling on."""
    op.profile_enable(True)
    _solve(op, s, B, **kw)
    n = sum(op.profile_read(c)[1] for c in ((cls,) if isinstance(cls, str) else cls))
    op.profile_enable(False)
    return n


_CONTRACT = ("contract_last", "contract_mid", "contract_rows")


def test_resident_batched_kernel_schedule():
    """Several small one-term two-mode systems: the resident kernel, replacing at once (chunks of one)."""
    from gpu_util import make_op, pack, unpack, infos
    import torch
    rng = np.random.default_rng(7001)
    systems = [wl.random_system(rng, dims, nterms=1, diag=diag, sigma2=0.2)
               for dims, diag in (((12, 10), True), ((9, 16), False), ((20, 7), True))]
    nrhs, tol = 2, 1e-10
    Bs = [rng.standard_normal((nrhs, s.n)) for s in systems]
    op = make_op(systems, prec="fp32")
    kw = dict(tol=tol, max_iters=2000, inner_tol=0.1, check_every=8)
    X, info = op.solve(pack(Bs), nrhs, prec="fp32", **kw)
    torch.cuda.synchronize()
    Xs = unpack(X, systems, nrhs)
    recs = infos(info, len(systems) * nrhs)
    op.profile_enable(True)
    op.solve(pack(Bs), nrhs, prec="fp32", **kw)
    torch.cuda.synchronize()
    _, n_res = op.profile_read("resident")
    op.profile_enable(False)
    op.close()
    assert n_res >= 1
    for k, s in enumerate(systems):
        ref = _oracle(s, Bs[k], tol, 0.1, 1, 2000)
        _compare(s, Bs[k], Xs[k], recs[k * nrhs:(k + 1) * nrhs], ref, tol, iter_band=3)


@pytest.mark.parametrize("every", [1, 4])
def test_general_path_schedule_small(every):
    """One two-term two-mode system with a diagonal on the contraction passes, chunks of `every`."""
    from gpu_util import make_op
    rng = np.random.default_rng(7002)
    s = wl.random_system(rng, (12, 10), nterms=2, diag=True, sigma2=0.2)
    B = rng.standard_normal((3, s.n))
    tol = 1e-10
    op = make_op([s], prec="fp32")
    kw = dict(tol=tol, max_iters=2000, inner_tol=0.1, check_every=every)
    X, rec = _solve(op, s, B, **kw)
    n_upd = _launches(op, s, B, "update", **kw)
    n_res64 = _launches(op, s, B, tuple(c + "_fp64" for c in _CONTRACT), **kw)
    n_res = _launches(op, s, B, "resident", **kw)
    op.close()
    assert n_upd >= 1 and n_res64 >= 1 and n_res == 0
    _compare(s, B, X, rec, _oracle(s, B, tol, 0.1, every, 2000), tol, iter_band=3)


# 64^3 one-term Wishart operator (condition number about 700, some 230 iterations to 1e-8): the
# persistent fused CG with host-polled chunks of 16 and with the device-side chunks of 128 that
# need no host wait (check_every = 0), the slab kernels with their device-side chunks of 32, and
# the plain contraction passes with chunks of 16.
_W64 = {}


def _w64():
    if not _W64:
        rng = np.random.default_rng(7003)
        s = wl.random_system(rng, (64, 64, 64), nterms=1, diag=False, sigma2=0.1)
        _W64["sys"] = s
        _W64["B"] = rng.standard_normal((2, s.n))
    return _W64["sys"], _W64["B"]


@pytest.mark.parametrize("engine,every,chunk,cls", [("fused", 16, 16, "cg_fused"), ("fused", 0, 128, "cg_fused"),
                                                    ("slab", 0, 32, "slab23"), ("contract", 16, 16, _CONTRACT)])
def test_schedule_64cube(engine, every, chunk, cls):
    from gpu_util import make_op
    s, B = _w64()
    tol = 1e-8
    key = ("ref", chunk)
    if key not in _W64:
        _W64[key] = _oracle(s, B, tol, 0.1, chunk, 3000)
    op = make_op([s], prec="fp32")
    if engine != "fused":
        op.set_engine("fused_cg", False)
    if engine == "contract":
        op.set_engine("slab", False)
    kw = dict(tol=tol, max_iters=3000, inner_tol=0.1, check_every=every)
    X, rec = _solve(op, s, B, **kw)
    n = _launches(op, s, B, cls, **kw)
    op.close()
    assert n >= 1, (engine, cls)
    _compare(s, B, X, rec, _W64[key], tol, iter_band=6)


def _refine_oracle(s, B, tol, inner_tol, max_sweeps, max_iters):
    A64 = lambda V: kron.mvm(s.factors, V, s.sigma2, s.diag)
    return ocg.refine(A64, _low(s), B, tol=tol, inner_tol=inner_tol, max_sweeps=max_sweeps,
                      inner_max_iters=max_iters)


def _compare_refine(s, B, X, rec, ref, tol, iter_band):
    rr = kron.relres(s.factors, X, B, s.sigma2, s.diag)
    kappa = _cond(s)
    for i in range(B.shape[0]):
        assert rec[i]["status"] == 0 and ref.status[i] == "ok", (rec[i], ref.status[i])
        assert rec[i]["sweeps"] == int(ref.sweeps[i]), (i, rec[i], ref.sweeps)
        assert abs(rec[i]["iters"] - int(ref.inner_iters[i])) <= iter_band, (i, rec[i], ref.inner_iters)
        assert rr[i] <= tol and abs(rec[i]["relres_true"] - rr[i]) <= 1e-3 * rr[i], (rr, rec[i])
        xn = np.linalg.norm(ref.X[i])
        assert np.linalg.norm(X[i] - ref.X[i]) <= 4.0 * kappa * tol * xn, (i, kappa)


@pytest.mark.parametrize("inner_tol", [1e-2, 1e-3, 1e-5])
def test_restart_schedule_small(inner_tol):
    """Two-term two-mode system with a diagonal on the contraction passes (4-8 sweeps of ~10-25
    inner iterations)."""
    from gpu_util import make_op
    rng = np.random.default_rng(7002)
    s = wl.random_system(rng, (12, 10), nterms=2, diag=True, sigma2=0.2)
    B = rng.standard_normal((3, s.n))
    tol = 1e-10
    op = make_op([s], prec="fp32")
    kw = dict(tol=tol, max_iters=3000, inner_tol=inner_tol, max_sweeps=20, check_every=4, refine="restart")
    X, rec = _solve(op, s, B, **kw)
    op.close()
    _compare_refine(s, B, X, rec, _refine_oracle(s, B, tol, inner_tol, 20, 3000), tol, iter_band=3)


def test_restart_schedule_64cube_fused():
    """The 64^3 Wishart operator on the persistent fused CG (inner solves without reliable updates):
    3 sweeps of ~90 inner iterations to 1e-8."""
    from gpu_util import make_op
    s, B = _w64()
    tol, inner_tol = 1e-8, 1e-3
    key = ("refine", inner_tol)
    if key not in _W64:
        _W64[key] = _refine_oracle(s, B, tol, inner_tol, 20, 3000)
    op = make_op([s], prec="fp32")
    kw = dict(tol=tol, max_iters=3000, inner_tol=inner_tol, max_sweeps=20, check_every=16, refine="restart")
    X, rec = _solve(op, s, B, **kw)
    n = _launches(op, s, B, "cg_fused", **kw)
    op.close()
    assert n >= 1
    _compare_refine(s, B, X, rec, _W64[key], tol, iter_band=6)


def _bf16_two_gemm_low(s):
    """The BF16 two-GEMM engine's product as the oracle emulates it: BF16 factors, the direction's
    BF16 copy in the first GEMM, its output T rounded to BF16 before the second, the diagonal term
    on the FP32 direction; sums in FP64 (the engine's FP32 accumulation order is the difference)."""
    n1, n2 = (f.shape[0] for f in s.factors[0])
    U = [lowprec.to_bf16(row[0]) for row in s.factors]
    V = [lowprec.to_bf16(row[1]) for row in s.factors]
    dd = float(np.float32(s.sigma2)) + (0.0 if s.diag is None else lowprec.to_fp32(s.diag))

    def apply(P):
        out = np.empty_like(P)
        P16 = lowprec.to_bf16(P)
        for i in range(P.shape[0]):
            X = P16[i].reshape(n1, n2)
            y = sum(u @ lowprec.to_bf16(X @ v.T) for u, v in zip(U, V))
            out[i] = y.reshape(-1) + dd * P[i]
        return out
    return apply


@pytest.mark.parametrize("every", [8, 32])
def test_bf16_restart_direction_schedule(every):
    """Plain BF16 working precision restarts the direction at every replacement (the rounded
    operator is too coarse for the old one): the two-GEMM engine against oracle.cg.reliable with
    restart_dir and the engine's roundings emulated (52-84 iterations, 4-7 replacements)."""
    from gpu_util import make_op
    rng = np.random.default_rng(7010)
    s = wl.random_system(rng, (256, 256), nterms=2, diag=True, sigma2=0.3)
    B = rng.standard_normal((2, s.n))
    tol = 1e-8
    op = make_op([s], prec="bf16")
    kw = dict(tol=tol, max_iters=2000, inner_tol=0.1, check_every=every)
    import torch
    from gpu_util import infos, pack, unpack
    X, info = op.solve(pack([B]), 2, prec="bf16", **kw)
    torch.cuda.synchronize()
    X, rec = unpack(X, [s], 2)[0], infos(info, 2)
    n = _launches_prec(op, s, B, "gemm_mode1", "bf16", **kw)
    op.close()
    assert n >= 1
    A64 = lambda V: kron.mvm(s.factors, V, s.sigma2, s.diag)
    ref = ocg.reliable(A64, _bf16_two_gemm_low(s), B, tol=tol, delta=0.1, max_iters=2000, check_every=every,
                       restart_dir=True)
    _compare(s, B, X, rec, ref, tol, iter_band=3)


def _launches_prec(op, s, B, cls, prec, **kw):
    import torch
    from gpu_util import pack
    op.profile_enable(True)
    op.solve(pack([B]), B.shape[0], prec=prec, **kw)
    torch.cuda.synchronize()
    n = sum(op.profile_read(c)[1] for c in ((cls,) if isinstance(cls, str) else cls))
    op.profile_enable(False)
    return n


def _bf16x3_contraction_low(s):
    """BF16x3 mode products as the oracle emulates them: every factor and every pass's input split
    three ways (v = h + m + l, each part the BF16 rounding of the remainder), the six leading cross
    products summed, each pass's output rounded to FP32, modes from the last to the first."""
    dims = [f.shape[0] for f in s.factors[0]]
    F = [[lowprec.bf16_split(f, 3) for f in row] for row in s.factors]
    dd = float(np.float32(s.sigma2)) + (0.0 if s.diag is None else lowprec.to_fp32(s.diag))

    def mode(T, parts, k):
        tp = lowprec.bf16_split(T, 3)
        out = 0.0
        for fi in range(3):
            for ti in range(3 - fi):
                out = out + np.moveaxis(np.tensordot(tp[ti], parts[fi], axes=([k + 1], [1])), -1, k + 1)
        return lowprec.to_fp32(out)

    def apply(P):
        out = np.zeros_like(P)
        for row in F:
            T = P.reshape((P.shape[0],) + tuple(dims))
            for k in reversed(range(len(dims))):
                T = mode(T, row[k], k)
            out += T.reshape(P.shape[0], -1)
        return out + dd * P
    return apply


@pytest.mark.parametrize("every", [1, 16])
def test_bf16x3_schedule_contraction_passes(every):
    """BF16x3 working precision on the general contraction passes (a 40 x 36 x 32 operator with a
    diagonal, ~140 iterations to 1e-9) against oracle.cg.reliable with the split products emulated."""
    from gpu_util import make_op
    rng = np.random.default_rng(7020)
    s = wl.random_system(rng, (40, 36, 32), nterms=1, diag=True, sigma2=0.1)
    B = rng.standard_normal((2, s.n))
    tol = 1e-9
    op = make_op([s], prec="bf16x3")
    kw = dict(tol=tol, max_iters=3000, inner_tol=0.1, check_every=every)
    import torch
    from gpu_util import infos, pack, unpack
    X, info = op.solve(pack([B]), 2, prec="bf16x3", **kw)
    torch.cuda.synchronize()
    X, rec = unpack(X, [s], 2)[0], infos(info, 2)
    n = _launches_prec(op, s, B, _CONTRACT, "bf16x3", **kw)
    op.close()
    assert n >= 1
    A64 = lambda V: kron.mvm(s.factors, V, s.sigma2, s.diag)
    ref = ocg.reliable(A64, _bf16x3_contraction_low(s), B, tol=tol, delta=0.1, max_iters=3000, check_every=every)
    _compare(s, B, X, rec, ref, tol, iter_band=4)
