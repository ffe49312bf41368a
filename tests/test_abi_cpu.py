"""The C ABI library loads and exports every symbol include/cola.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cola.h")
LIB = os.path.join(ROOT, "paper_2309_03060_amd", "libcola.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cola_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("cola_op_create", "cola_op_destroy", "cola_kron_matvec", "cola_cg_solve",
                     "cola_cg_solve_backward", "cola_status_string"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcola.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcola.so not built")
def test_status_strings_and_null_argument_errors():
    from paper_2309_03060_amd import _lib as L
    lib = L.lib()
    assert L.status_string(L.COLA_OK) == "ok"
    assert "positive definite" in L.status_string(L.COLA_ERR_NOT_SPD)
    assert L.status_string(12345) == "unknown status"
    # argument validation happens before any device call
    out = ctypes.c_void_p()
    assert lib.cola_op_create(None, 1, 0, None, ctypes.byref(out)) == L.COLA_ERR_INVALID_ARG
    assert lib.cola_op_create(None, 1, 0, None, None) == L.COLA_ERR_INVALID_ARG
    assert lib.cola_op_destroy(None) == L.COLA_OK
    assert lib.cola_kron_matvec(None, None, None, 1, 0, 0, None) == L.COLA_ERR_INVALID_ARG
    assert lib.cola_kron_matvec_noalloc(None, None, None, 1, 0, 0, None) == L.COLA_ERR_INVALID_ARG
    assert "scratch" in L.status_string(L.COLA_ERR_SCRATCH)
    assert lib.cola_cg_solve(None, None, None, 1, None, None, None) == L.COLA_ERR_INVALID_ARG
    assert lib.cola_cg_solve_backward(None, None, None, 1, None, None, None, None, None, None, None) == \
        L.COLA_ERR_INVALID_ARG
    assert lib.cola_op_size(None, None, None) == L.COLA_ERR_INVALID_ARG
    # bad descriptor fields are rejected before any allocation
    d = L.SystemDesc()
    d.nterms, d.nfactors = 1, 4
    assert lib.cola_op_create(ctypes.byref(d), 1, 0, None, ctypes.byref(out)) == L.COLA_ERR_INVALID_ARG
    d.nfactors = 2
    d.dims[0], d.dims[1] = 3, 0
    arr = (ctypes.c_void_p * 2)(1, 1)
    d.factors = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
    assert lib.cola_op_create(ctypes.byref(d), 1, 0, None, ctypes.byref(out)) == L.COLA_ERR_INVALID_ARG
    d.dims[1] = 3
    d.sigma2 = float("nan")
    assert lib.cola_op_create(ctypes.byref(d), 1, 0, None, ctypes.byref(out)) == L.COLA_ERR_INVALID_ARG
    d.sigma2 = 0.1
    assert lib.cola_op_create(ctypes.byref(d), 1, 7, None, ctypes.byref(out)) == L.COLA_ERR_INVALID_ARG


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2309_03060_amd import _lib as L
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(RuntimeError, match="not found"):
        L.lib()
