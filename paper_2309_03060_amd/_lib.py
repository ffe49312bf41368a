"""ctypes binding of libcola (include/cola.h): argument marshalling only.

Names mirror the C entry points.  Loading fails loudly when the HIP library
has not been built: there is no CPU fallback anywhere in this package.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcola.so")

COLA_OK = 0
COLA_NOT_CONVERGED = 1
COLA_STAGNATED = 2
COLA_ERR_INVALID_ARG = -1
COLA_ERR_NOT_SPD = -2
COLA_ERR_NONFINITE = -3
COLA_ERR_OOM = -4
COLA_ERR_HIP = -5
COLA_ERR_UNSUPPORTED = -6
COLA_ERR_SCRATCH = -7

COLA_F64 = 0
COLA_F32 = 1

COLA_PREC_FP64 = 0
COLA_PREC_FP32 = 1
COLA_PREC_BF16 = 2
COLA_PREC_BF16X3 = 3

COLA_REFINE_RELIABLE = 0
COLA_REFINE_RESTART = 1
REFINE_BY_NAME = {"reliable": COLA_REFINE_RELIABLE, "restart": COLA_REFINE_RESTART}

ENGINE_BY_NAME = {"fused_cg": 1, "gemm2": 2, "gemm3": 3, "slab": 4, "resident": 5, "small64": 6, "gemm64": 7}
PRECOND_BY_NAME = {"none": 0, "jacobi": 1, "kron_eig": 2}
DIAG_MODE_BY_NAME = {"hutchinson": 0, "doubly": 1}

PREC_BY_NAME = {"fp64": COLA_PREC_FP64, "fp32": COLA_PREC_FP32,
                "bf16": COLA_PREC_BF16, "bf16x3": COLA_PREC_BF16X3}

EXPORTED = ("cola_op_create", "cola_op_destroy", "cola_op_memory", "cola_op_size", "cola_kron_matvec",
            "cola_kron_matvec_noalloc",
            "cola_op_diagonal", "cola_diag_estimate",
            "cola_cg_solve", "cola_cg_solve_backward", "cola_logdet_grad", "cola_eig_solve", "cola_slq_logdet",
            "cola_autotune", "cola_autotune_export", "cola_autotune_import",
            "cola_op_set_engine", "cola_profile_enable", "cola_profile_read", "cola_trace_enable",
            "cola_status_string")


class SystemDesc(ctypes.Structure):
    _fields_ = [("nterms", ctypes.c_int32), ("nfactors", ctypes.c_int32),
                ("dims", ctypes.c_int64 * 3), ("factors", ctypes.POINTER(ctypes.c_void_p)),
                ("diag", ctypes.c_void_p), ("sigma2", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iters", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("max_sweeps", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("refine", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("x0_given", ctypes.c_int32), ("hist_stride", ctypes.c_int32), ("hist_len", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("hist", ctypes.c_void_p)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("relres_recursive", ctypes.c_double),
                ("relres_true", ctypes.c_double)]


INFO_WORDS = ctypes.sizeof(SolveInfo) // 4      # int32 words per cola_solve_info record


class ColaError(RuntimeError):
    def __init__(self, call: str, status: int):
        self.status = status
        super().__init__(f"{call} failed: {status_string(status)} ({status})")


_lib = None


def lib():
    """The loaded library; raises if it is missing (build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libcola.so not found at {LIB_PATH}: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.cola_op_create.argtypes = [ctypes.POINTER(SystemDesc), i32, i32, vp, ctypes.POINTER(vp)]
        L.cola_op_destroy.argtypes = [vp]
        L.cola_op_memory.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), i32]
        L.cola_op_size.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32)]
        L.cola_kron_matvec.argtypes = [vp, vp, vp, i32, i32, i32, vp]
        L.cola_kron_matvec_noalloc.argtypes = [vp, vp, vp, i32, i32, i32, vp]
        L.cola_cg_solve.argtypes = [vp, vp, vp, i32, ctypes.POINTER(SolveOpts), vp, vp]
        L.cola_cg_solve_backward.argtypes = [vp, vp, vp, i32, ctypes.POINTER(SolveOpts), vp,
                                             ctypes.POINTER(vp), ctypes.POINTER(vp), vp, vp, vp]
        L.cola_logdet_grad.argtypes = [vp, vp, i32, ctypes.POINTER(SolveOpts), vp, ctypes.POINTER(vp),
                                       ctypes.POINTER(vp), vp, vp, vp]
        L.cola_eig_solve.argtypes = [vp, vp, vp, i32, vp]
        L.cola_op_diagonal.argtypes = [vp, vp, vp]
        L.cola_diag_estimate.argtypes = [vp, vp, i32, i32, vp, vp]
        L.cola_slq_logdet.argtypes = [vp, vp, i32, dbl, i32, vp, vp, vp, vp, vp]
        L.cola_autotune.argtypes = [vp, i32, vp]
        L.cola_op_set_engine.argtypes = [vp, i32, i32]
        L.cola_profile_enable.argtypes = [vp, i32]
        L.cola_trace_enable.argtypes = [i32]
        L.cola_autotune_export.argtypes = [vp, ctypes.c_char_p, i64, ctypes.POINTER(i64)]
        L.cola_autotune_import.argtypes = [vp, ctypes.c_char_p]
        L.cola_profile_read.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
        L.cola_status_string.argtypes = [i32]
        L.cola_status_string.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name != "cola_status_string":
                getattr(L, name).restype = i32
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().cola_status_string(int(status)).decode()


def check(call: str, status: int) -> None:
    if status != COLA_OK:
        raise ColaError(call, status)
