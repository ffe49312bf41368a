"""Sum-of-Kronecker-plus-diagonal CG on MI355X (gfx950): Python binding.

The work is done by libcola.so (HIP kernels behind the C ABI in
include/cola.h).  This package only marshals arguments; importing it does
not load the library, and every entry point fails loudly when the library
is missing.
"""
from ._lib import (COLA_OK, COLA_NOT_CONVERGED, COLA_STAGNATED, COLA_ERR_NOT_SPD,  # noqa: F401
                   COLA_ERR_NONFINITE, COLA_ERR_INVALID_ARG, ColaError, status_string, lib)
from .ops import KronOperator, SystemSpec, KronSolve, kron_cg_solve, decode_info  # noqa: F401
