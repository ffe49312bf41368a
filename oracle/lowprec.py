"""Rounding emulator for bfloat16 / float32 working copies (diagnostic).

App. C.3 motivates lower-precision solves and notes that round-off is what
breaks numerical linear algebra routines; it gives no scheme.  This module
rounds float64 data the way the GPU's conversions do, so each workload's
working precision can be checked for positive definiteness before any
kernel runs:

* bf16: round to nearest, ties to even, on the float32 bit pattern
  (1 sign, 8 exponent, 7 stored mantissa bits);
* bf16 x k split: v ~ h1 + h2 + ... + hk with each h_i the bf16 rounding of
  what the previous parts leave over.

TEST INFRASTRUCTURE: see the package docstring.
"""
from __future__ import annotations

import numpy as np


def to_bf16(v: np.ndarray) -> np.ndarray:
    """Round (via float32) to bfloat16, ties to even; returned as float64."""
    f = np.ascontiguousarray(np.asarray(v, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def to_fp32(v: np.ndarray) -> np.ndarray:
    return np.asarray(v, dtype=np.float64).astype(np.float32).astype(np.float64)


def bf16_split(v: np.ndarray, parts: int):
    """Split v into `parts` bf16 pieces, each the rounding of the remainder."""
    rest = to_fp32(v)
    out = []
    for _ in range(parts):
        h = to_bf16(rest)
        out.append(h)
        rest = to_fp32(rest - h)
    return out


def bf16_split_value(v: np.ndarray, parts: int) -> np.ndarray:
    return sum(bf16_split(v, parts))


def min_eig_rounded(factors, sigma2: float, rounder) -> float:
    """Smallest eigenvalue of (x)_k round(K_k) + sigma2 I (one Kronecker term).

    By the Kronecker eigenvalue rule the spectrum is all products of the
    rounded factors' eigenvalues; the minimum is taken over those products.
    """
    lam = np.array([1.0])
    for f in factors:
        r = rounder(np.asarray(f, dtype=np.float64))
        w = np.linalg.eigvals(r).real
        lam = np.kron(lam, w)
    return float(lam.min() + sigma2)
