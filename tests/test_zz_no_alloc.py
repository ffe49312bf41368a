"""The no-allocation product (cola_kron_matvec_noalloc) against cola_kron_matvec, through the C ABI.

Two calls in a row on one op, the second with fewer right-hand sides, per working precision and
engine family (general contraction passes with the fused mode-2/3 slab, FP64 passes, the BF16
two-GEMM engine).  The two entry points run the same kernels on the same data with the
intermediates in different buffers, so the products must agree bit for bit; each is also held to
the oracle's product at its precision's tolerance.  A fresh op's device memory must not grow (its
workspace is never allocated), and a call too large for the static scratch is refused before
anything is enqueued.
"""
import ctypes

import numpy as np
import pytest

import workloads as wl
from oracle import kron, lowprec

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-13, "fp32": 2e-6, "bf16": 2e-2}


def _systems(kind, rng):
    if kind == "bf16":
        return [wl.random_system(rng, (256, 512), nterms=3, diag=True, sigma2=0.3)]
    return [wl.random_system(rng, (40, 36, 20), nterms=1, diag=True, sigma2=0.2),
            wl.random_system(rng, (33, 17), nterms=2, diag=True, sigma2=0.1),
            wl.random_system(rng, (7,), nterms=1, diag=False, sigma2=0.4)]


def _noalloc(op, X, Y, nrhs, prec):
    from paper_2309_03060_amd import _lib as L
    from paper_2309_03060_amd.ops import _stream_ptr
    p = L.PREC_BY_NAME[prec]
    dtype = L.COLA_F64 if p == L.COLA_PREC_FP64 else L.COLA_F32
    return op.lib.cola_kron_matvec_noalloc(op.handle, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                                          nrhs, dtype, p, ctypes.c_void_p(_stream_ptr()))


@pytest.mark.parametrize("op_prec,prec", [("fp32", "fp32"), ("fp32", "fp64"), ("bf16", "bf16")])
def test_noalloc_matches_matvec_two_calls(op_prec, prec):
    import torch
    from gpu_util import make_op, pack, unpack
    rng = np.random.default_rng(71)
    systems = _systems(op_prec, rng)
    op = make_op(systems, prec=op_prec)
    dt = torch.float64 if prec == "fp64" else torch.float32
    for nrhs in (3, 1):                                   # the second call is smaller
        Xs = [rng.standard_normal((nrhs, s.n)) for s in systems]
        X = pack(Xs, dt)
        Yn = torch.full_like(X, float("nan"))
        torch.cuda.synchronize()
        live0 = op.memory()[0]                            # the first pass: a fresh op, no workspace yet
        assert _noalloc(op, X, Yn, nrhs, prec) == 0
        torch.cuda.synchronize()
        assert op.memory()[0] == live0                    # nothing allocated by the library
        Yr = op.matvec(X, nrhs, prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(Yn, Yr), (nrhs, float((Yn - Yr).abs().max()))
        for s, Xk, Yk in zip(systems, Xs, unpack(Yn, systems, nrhs)):
            Xq = Xk if prec == "fp64" else lowprec.to_fp32(Xk)
            ref = kron.mvm(s.factors, Xq, s.sigma2, s.diag)
            absref = kron.mvm([[np.abs(f) for f in row] for row in s.factors], np.abs(Xq), abs(s.sigma2),
                              None if s.diag is None else np.abs(s.diag))
            assert (np.abs(Yk - ref) / absref).max() <= TOL[prec]
    op.close()


def test_noalloc_refuses_calls_beyond_its_scratch():
    """A 256^3 operator needs 64 MiB per intermediate for one right-hand side: refused with
    COLA_ERR_SCRATCH, nothing enqueued (the output keeps its contents)."""
    import torch
    from paper_2309_03060_amd import _lib as L
    from gpu_util import make_op
    rng = np.random.default_rng(72)
    s = wl.random_system(rng, (256, 256, 256), nterms=1, diag=False, sigma2=0.5)
    op = make_op([s], prec="bf16x3")
    X = torch.ones(s.n, dtype=torch.float32, device="cuda:0")
    Y = torch.full_like(X, 7.0)
    assert _noalloc(op, X, Y, 1, "bf16x3") == L.COLA_ERR_SCRATCH
    torch.cuda.synchronize()
    assert bool((Y == 7.0).all())
    assert "scratch" in L.status_string(L.COLA_ERR_SCRATCH)
    op.close()
