"""Forward solve + adjoint backward captured in one HIP graph and replayed.

With check_every = 0 the library never waits on the host, allocates nothing
after the first call for a given nrhs, and records no memset, so the whole
sequence can be captured.  Every replay is checked against the eager result,
with eager work and synchronisations between replays.
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _capture_and_replay(systems, Bs, Ws, nrhs, prec, kw, replays=3, check_eager=None):
    import torch
    from gpu_util import make_op, pack
    op = make_op(systems, prec=prec)
    B = pack(Bs)
    G = pack(Ws)
    # eager reference (also sizes the workspace)
    X_e, _ = op.solve(B, nrhs, **kw)
    if check_eager is not None:
        check_eager(op, B, X_e)
    Lam_e, dfac_e, _, ds2_e, _ = op.solve_backward(X_e, G, nrhs, **kw)
    torch.cuda.synchronize()
    ref = (X_e.clone(), Lam_e.clone(), [t.clone() for s in dfac_e for row in s for t in row], ds2_e.clone())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        X_g, _ = op.solve(B, nrhs, **kw)
        Lam_g, dfac_g, _, ds2_g, _ = op.solve_backward(X_g, G, nrhs, **kw)
    for rep in range(replays):
        X_g.zero_()
        Lam_g.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(X_g, ref[0]), rep
        assert torch.equal(Lam_g, ref[1]), rep
        got = [t for s in dfac_g for row in s for t in row]
        for a, b in zip(got, ref[2]):
            assert torch.equal(a, b), rep
        assert torch.equal(ds2_g, ref[3]), rep
        # eager work between replays
        X_x, _ = op.solve(B, nrhs, **kw)
        torch.cuda.synchronize()
        assert torch.equal(X_x, ref[0])
    op.close()


def test_graph_replay_streaming_path_matches_eager():
    w = wl.config2(m=12, nrhs=2)
    rng = np.random.default_rng(71)
    Ws = [rng.standard_normal(w.B[0].shape)]
    _capture_and_replay(w.systems, w.B, Ws, 2, "fp32", dict(tol=1e-8, max_iters=256, check_every=0))


def test_graph_replay_uneven_batch_matches_eager():
    w = wl.config3(nsys=8, dmin=16, dmax=64, seed=72)
    _capture_and_replay(w.systems, w.B, w.W, 1, "fp32", dict(tol=1e-8, max_iters=2000, check_every=0))


def test_graph_replay_fused_engine_matches_eager():
    """64^3 RBF operator (the persistent fused CG's shape), FP32 with FP64 reliable updates,
    check_every = 0: every 128-iteration cooperative launch and reliable-update tail is enqueued up
    front, captured together with the backward and replayed bit-exactly.  The eager solve took the
    fused engine (its launches counted) and equals, bit for bit, the host-checked solve with the same
    128-iteration chunks."""
    import torch
    w = wl.config2(m=64, nrhs=2)
    rng = np.random.default_rng(73)
    Ws = [rng.standard_normal(w.B[0].shape)]
    kw = dict(tol=1e-8, max_iters=300, check_every=0)

    def fused_ran(op, B, X_e):
        op.profile_enable(True)
        X0, info0 = op.solve(B, 2, **kw)
        torch.cuda.synchronize()
        _, launches = op.profile_read("cg_fused")
        op.profile_enable(False)
        assert launches >= 3, launches                    # ceil(300 / 128) chunks
        X1, _ = op.solve(B, 2, **dict(kw, check_every=128))
        torch.cuda.synchronize()
        assert torch.equal(X0, X_e) and torch.equal(X1, X_e)

    _capture_and_replay(w.systems, w.B, Ws, 2, "fp32", kw, check_eager=fused_ran)
