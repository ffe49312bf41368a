"""The tuning cache: a tile table exported by one op and imported by another of the same shapes.

A miss tunes and writes the table (a device line and one line per tuned pass); a second op of the
same shapes hits, loads exactly those tiles, and produces bit-identical solves; a table of another
device is read and ignored; a malformed line is refused with nothing applied.
"""
import json

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def test_tuning_cache_round_trip(tmp_path):
    import ctypes

    import torch
    from gpu_util import make_op, pack
    from paper_2309_03060_amd import _lib as L
    rng = np.random.default_rng(31)
    s = wl.random_system(rng, (40, 36, 24), nterms=2, diag=True, sigma2=0.2)
    B = rng.standard_normal((2, s.n))
    cache = str(tmp_path / "tiles.json")

    def table(op):
        n = ctypes.c_int64()
        assert op.lib.cola_autotune_export(op.handle, None, 0, ctypes.byref(n)) == 0
        buf = ctypes.create_string_buffer(n.value + 1)
        assert op.lib.cola_autotune_export(op.handle, buf, n.value + 1, ctypes.byref(n)) == 0
        return buf.value.decode()

    op1 = make_op([s], prec="fp32")
    assert op1.autotune(2, cache=cache) is False              # miss: tuned and stored
    t1 = table(op1)
    lines = t1.strip().splitlines()
    assert lines[0].startswith("device gfx950 ") and len(lines) >= 4
    stored = json.load(open(cache))
    assert list(stored.values()) == [t1]
    X1, _ = op1.solve(pack([B]), 2, tol=1e-9, max_iters=500, prec="fp32")
    op2 = make_op([s], prec="fp32")
    assert op2.autotune(2, cache=cache) is True               # hit: loaded, not timed
    assert table(op2) == t1
    X2, _ = op2.solve(pack([B]), 2, tol=1e-9, max_iters=500, prec="fp32")
    torch.cuda.synchronize()
    assert torch.equal(X1, X2)
    # another device's entries are read and ignored; malformed text is refused
    body = "\n".join(lines[1:])
    other = "device gfx000 8\n" + "\n".join(l.rsplit(" ", 2)[0] + " 1 1" for l in lines[1:]) + "\n"
    assert op2.lib.cola_autotune_import(op2.handle, other.encode()) == 0
    assert table(op2) == t1
    assert op2.lib.cola_autotune_import(op2.handle, (lines[0] + "\n1 0 40 1\n").encode()) == L.COLA_ERR_INVALID_ARG
    assert op2.lib.cola_autotune_import(op2.handle, (lines[0] + "\n" + body.replace(" ", " 3 ", 1)).encode()) \
        == L.COLA_ERR_INVALID_ARG
    assert table(op2) == t1
    op1.close()
    op2.close()
