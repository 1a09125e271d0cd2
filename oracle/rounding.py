"""Reduced-precision rounding used to emulate the GPU's GEMM inputs (FP64).

Test infrastructure only.  bfloat16: 8 significant bits, float32 exponent
range, round to nearest even.  E4M3FN (OCP 8-bit float): 4 significant bits,
exponent bias 7, smallest normal 2^-6, subnormal step 2^-9, largest finite
448, no infinities; here saturating to +-448.
"""
from __future__ import annotations

import numpy as np


def _round_sig(x, sig_bits, min_exp):
    """Round to ``sig_bits`` significant bits, ties to even, with gradual
    underflow below 2^min_exp.  Exact in float64 (power-of-two scalings)."""
    x = np.asarray(x, np.float64)
    ax = np.abs(x)
    # frexp is exact: ax = f * 2^ef with 0.5 <= f < 1
    _, ef = np.frexp(np.where(ax > 0, ax, 1.0))
    e = (ef - 1).astype(np.float64)
    e = np.maximum(e, min_exp)
    q = np.ldexp(1.0, (e - (sig_bits - 1)).astype(np.int64))
    return np.rint(x / q) * q


def round_bf16(x):
    """float64 -> nearest bfloat16 value (as float64), ties to even."""
    x = np.asarray(x, np.float64)
    r = _round_sig(x, 8, -126)
    big = (2.0 - 2.0 ** -8) * 2.0 ** 127
    r = np.where(np.abs(x) >= big, np.copysign(np.inf, x), r)
    return np.where(np.isnan(x), np.nan, r)


def round_e4m3(x):
    """float64 -> nearest E4M3FN value (as float64), ties to even, saturating."""
    x = np.asarray(x, np.float64)
    r = _round_sig(x, 4, -6)
    r = np.clip(r, -448.0, 448.0)
    return np.where(np.isnan(x), np.nan, r)
