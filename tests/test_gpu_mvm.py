"""GPU parity of cola_kron_matvec against the float64 oracle (element by element)."""
import numpy as np
import pytest

import workloads as wl
from oracle import kron, lowprec

pytestmark = pytest.mark.gpu

SHAPES = [
    ((7,), 1, False),            # single dense factor (F = 1)
    ((5, 7), 1, False),          # ragged, smaller than one tile
    ((33, 17), 2, True),         # crosses tile edges, two terms, diagonal
    ((64, 64), 1, False),        # whole tiles
    ((5, 7, 3), 1, True),        # three modes, ragged
    ((16, 8, 24), 3, False),     # three terms
    ((40, 36, 20), 1, True),     # several tiles per mode, ragged tails
    ((130, 70), 2, True),        # mode sizes above the largest tile
]


def _systems(shape, nterms, diag, seed=0):
    rng = np.random.default_rng(100 + seed)
    s = wl.random_system(rng, shape, nterms=nterms, diag=diag, sigma2=0.37)
    # non-symmetric factors catch a transposed operand
    s.factors = [[f + 0.05 * rng.standard_normal(f.shape) for f in row] for row in s.factors]
    return s


@pytest.mark.parametrize("shape,nterms,diag", SHAPES)
@pytest.mark.parametrize("nrhs", [1, 3])
def test_matvec_fp64(shape, nterms, diag, nrhs):
    import torch
    from gpu_util import make_op, pack, unpack
    s = _systems(shape, nterms, diag)
    X = np.random.default_rng(1).standard_normal((nrhs, s.n))
    op = make_op([s], prec="fp64")
    Y = unpack(op.matvec(pack([X]), nrhs, prec="fp64"), [s], nrhs)[0]
    ref = kron.mvm(s.factors, X, s.sigma2, s.diag)
    err = np.abs(Y - ref).max() / np.abs(ref).max()
    assert err <= 1e-13, err
    op.close()


@pytest.mark.parametrize("prec,tol", [("fp32", 2e-6), ("bf16x3", 4e-6), ("bf16", 2e-2)])
@pytest.mark.parametrize("shape,nterms,diag", SHAPES)
def test_matvec_low_precision(prec, tol, shape, nterms, diag):
    import torch
    from gpu_util import make_op, pack, unpack
    s = _systems(shape, nterms, diag, seed=1)
    nrhs = 2
    X = np.random.default_rng(2).standard_normal((nrhs, s.n))
    op = make_op([s], prec=prec)
    Y = unpack(op.matvec(pack([X], torch.float32), nrhs), [s], nrhs)[0]
    Xr = lowprec.to_fp32(X)
    ref = kron.mvm(s.factors, Xr, s.sigma2, s.diag)
    # error scale: |K| |x| products summed over each contraction
    absref = kron.mvm([[np.abs(f) for f in row] for row in s.factors], np.abs(Xr), abs(s.sigma2),
                      None if s.diag is None else np.abs(s.diag))
    err = (np.abs(Y - ref) / absref).max()
    assert err <= tol, err
    op.close()


def _bf16_rounded_mvm(s, X):
    """The oracle's product with every operand the BF16 path rounds rounded the same way (RNE via
    FP32): the factors, x, and each intermediate before its mode is multiplied; modes are applied
    last to first, as the passes do, and a single factor K acts as [1] (x) K (so its result is
    rounded once more before the trivial first mode).  The diagonal term uses the FP32 x and d."""
    dims = list(s.dims)
    terms = s.factors
    if len(dims) == 1:
        dims = [1] + dims
        terms = [[np.ones((1, 1))] + list(row) for row in terms]
    Xr = lowprec.to_fp32(X)
    Y = np.zeros_like(Xr)
    for row in terms:
        T = Xr
        for k in reversed(range(len(dims))):
            facs = [np.eye(d) for d in dims]
            facs[k] = lowprec.to_bf16(row[k])
            T = kron.kron_apply(facs, lowprec.to_bf16(T))
        Y += T
    dg = lowprec.to_fp32(np.full(s.n, s.sigma2) if s.diag is None else lowprec.to_fp32(s.diag) + s.sigma2)
    return Y + dg[None, :] * Xr


# BF16 against the oracle fed the same BF16 roundings: what remains is FP32 accumulation order and the
# rare BF16 rounding of an intermediate that FP32 accumulation pushes across a tie (one BF16 ulp of one
# element, ~2^-9 / n_k of the |K||x| scale).  Truncation instead of round-to-nearest-even, or a rounding
# point lost or added, moves every entry by ~1e-4 .. 1e-3 of that scale.
@pytest.mark.parametrize("shape,nterms,diag", SHAPES + [((256, 256), 1, False), ((256, 512), 3, True)])
def test_matvec_bf16_against_rounded_oracle(shape, nterms, diag):
    import torch
    from gpu_util import make_op, pack, unpack
    s = _systems(shape, nterms, diag, seed=1)
    nrhs = 2
    X = np.random.default_rng(2).standard_normal((nrhs, s.n))
    op = make_op([s], prec="bf16")
    Y = unpack(op.matvec(pack([X], torch.float32), nrhs), [s], nrhs)[0]
    op.close()
    ref = _bf16_rounded_mvm(s, X)
    Xr = lowprec.to_fp32(X)
    absref = kron.mvm([[np.abs(f) for f in row] for row in s.factors], np.abs(Xr), abs(s.sigma2),
                      None if s.diag is None else np.abs(s.diag))
    err = (np.abs(Y - ref) / absref).max()
    assert err <= 3e-5, err


def test_matvec_multi_system_packing():
    import torch
    from gpu_util import make_op, pack, unpack
    rng = np.random.default_rng(5)
    systems = [wl.random_system(rng, d, nterms=1, diag=(i % 2 == 0), sigma2=0.1 * i)
               for i, d in enumerate([(3, 4), (9, 2, 5), (17,), (20, 20)])]
    nrhs = 2
    Xs = [rng.standard_normal((nrhs, s.n)) for s in systems]
    op = make_op(systems, prec="fp64")
    Ys = unpack(op.matvec(pack(Xs), nrhs, prec="fp64"), systems, nrhs)
    for s, X, Y in zip(systems, Xs, Ys):
        ref = kron.mvm(s.factors, X, s.sigma2, s.diag)
        assert np.abs(Y - ref).max() <= 1e-13 * np.abs(ref).max()
    op.close()


def test_matvec_full_size_c2_sampled():
    """The bench workload's operator (64^3, 32 RHS): sampled entries against the oracle's definition."""
    import torch
    from gpu_util import make_op, pack, unpack
    w = wl.config2()
    s = w.systems[0]
    nrhs = 32
    X = w.B[0]
    op = make_op([s], prec="fp32")
    Y64 = unpack(op.matvec(pack([X]), nrhs, prec="fp64"), [s], nrhs)[0]
    Y32 = unpack(op.matvec(pack([X], torch.float32), nrhs), [s], nrhs)[0]
    rng = np.random.default_rng(9)
    for r in (0, 17, 31):
        for idx in rng.integers(0, s.n, size=6):
            ref = kron.mvm_entry(s.factors, X[r], int(idx), s.sigma2)
            scale = kron.mvm_entry([[np.abs(f) for f in s.factors[0]]], np.abs(X[r]), int(idx), s.sigma2)
            assert abs(Y64[r, idx] - ref) <= 1e-13 * scale
            assert abs(Y32[r, idx] - ref) <= 3e-6 * scale
    op.close()


# Two-mode operators whose modes are multiples of 256 run their BF16 MVM as two
# dense GEMMs (pack, mode-2 GEMM over all terms, mode-1 GEMM summing the terms).
GEMM_SHAPES = [((256, 256), 1, False, 1), ((256, 512), 3, True, 3), ((512, 256), 2, True, 2)]


@pytest.mark.parametrize("shape,nterms,diag,nrhs", GEMM_SHAPES)
def test_matvec_bf16_dense_gemm_path(shape, nterms, diag, nrhs):
    import torch
    from gpu_util import make_op, pack, unpack
    s = _systems(shape, nterms, diag, seed=3)
    X = np.random.default_rng(4).standard_normal((nrhs, s.n))
    op = make_op([s], prec="bf16")
    Y = unpack(op.matvec(pack([X], torch.float32), nrhs), [s], nrhs)[0]
    Xr = lowprec.to_fp32(X)
    ref = kron.mvm(s.factors, Xr, s.sigma2, s.diag)
    absref = kron.mvm([[np.abs(f) for f in row] for row in s.factors], np.abs(Xr), abs(s.sigma2),
                      None if s.diag is None else np.abs(s.diag))
    # BF16 operands and a BF16 intermediate: about four roundings of 2^-9 each
    err = (np.abs(Y - ref) / absref).max()
    assert err <= 2e-2, err
    # the same operator through the FP64 passes, for a tight structural check
    Y64 = unpack(op.matvec(pack([X]), nrhs, prec="fp64"), [s], nrhs)[0]
    assert np.abs(Y64 - kron.mvm(s.factors, X, s.sigma2, s.diag)).max() <= 1e-13 * np.abs(absref).max()
    op.close()


def test_matvec_bf16_gemm_path_after_unaligned_system():
    """A GEMM-shaped system packed after a small one (its vectors are not 16-byte aligned) still
    gives the right product (the contraction passes take over)."""
    import torch
    from gpu_util import make_op, pack, unpack
    rng = np.random.default_rng(6)
    systems = [wl.random_system(rng, (3, 5), nterms=1, diag=False, sigma2=0.2),
               wl.random_system(rng, (256, 256), nterms=2, diag=True, sigma2=0.1),
               wl.random_system(rng, (256, 256), nterms=1, diag=False, sigma2=0.3)]
    nrhs = 1
    Xs = [rng.standard_normal((nrhs, s.n)) for s in systems]
    op = make_op(systems, prec="bf16")
    Ys = unpack(op.matvec(pack(Xs, torch.float32), nrhs), systems, nrhs)
    for s, X, Y in zip(systems, Xs, Ys):
        Xr = lowprec.to_fp32(X)
        ref = kron.mvm(s.factors, Xr, s.sigma2, s.diag)
        absref = kron.mvm([[np.abs(f) for f in row] for row in s.factors], np.abs(Xr), abs(s.sigma2),
                          None if s.diag is None else np.abs(s.diag))
        assert (np.abs(Y - ref) / absref).max() <= 2e-2
    op.close()


# One-term three-mode operators with 256-wide modes run their FP32 and BF16x3 MVMs as
# three dense GEMMs (each pass writes its output with the new mode first); BF16x3
# splits every operand three ways and sums six BF16 matrix-core products.
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("shape,diag,nrhs", [((256, 256, 256), True, 2), ((512, 256, 256), False, 1),
                                             ((256, 512, 256), True, 3)])
def test_matvec_dense_gemm3_path(shape, diag, nrhs, prec):
    import torch
    from gpu_util import make_op, pack, unpack
    s = _systems(shape, 1, diag, seed=7)
    X = np.random.default_rng(8).standard_normal((nrhs, s.n))
    op = make_op([s], prec=prec)
    Y = unpack(op.matvec(pack([X], torch.float32), nrhs), [s], nrhs)[0]
    Xr = lowprec.to_fp32(X)
    ref = kron.mvm(s.factors, Xr, s.sigma2, s.diag)
    absref = kron.mvm([[np.abs(f) for f in row] for row in s.factors], np.abs(Xr), abs(s.sigma2),
                      None if s.diag is None else np.abs(s.diag))
    # three FP32-accumulated contractions of length 256 and 512; for BF16x3 the dropped products
    # (mid x lo, lo x mid, lo x lo) are about 2 * 2^-24 of each term.  A missing leading product
    # (hh alone: ~2^-9; without hl / lh / mm: ~2^-17) fails this bound.
    err = (np.abs(Y - ref) / absref).max()
    assert err <= 2e-6, err
    if prec == "bf16x3":
        # the same splits through the general contraction passes (engine off): the same six
        # products in another order, so the two agree to FP32 accumulation rounding
        op.set_engine("gemm3", False)
        Yc = unpack(op.matvec(pack([X], torch.float32), nrhs), [s], nrhs)[0]
        assert (np.abs(Y - Yc) / absref).max() <= 2e-6
    op.close()
