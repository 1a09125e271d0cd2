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


def _rounding_margin(x, sig_bits, min_exp):
    """Distance from x to the nearest rounding boundary (midpoint between two
    adjacent representable values) of a format with ``sig_bits`` significant
    bits and smallest normal exponent ``min_exp``, relative to |x|.  Within the
    binade [2^e, 2^(e+1)) of x (e at least min_exp) the representable values
    are multiples of q = 2^(e - sig_bits + 1), so the boundaries there are the
    odd multiples of q / 2; below 2^e the spacing halves, so the next boundary
    down is 2^e - q / 4.  Exact in float64 (power-of-two scalings)."""
    x = np.abs(np.asarray(x, np.float64))
    _, ef = np.frexp(np.where(x > 0, x, 1.0))
    e = np.maximum((ef - 1).astype(np.float64), min_exp)
    q = np.ldexp(1.0, (e - (sig_bits - 1)).astype(np.int64))
    u = x / q
    dist = np.abs(u - np.floor(u) - 0.5) * q
    low = np.ldexp(1.0, e.astype(np.int64))
    below = np.where(e > min_exp, x - (low - q / 4), np.inf)
    dist = np.minimum(dist, below)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(x > 0, dist / np.where(x > 0, x, 1.0), np.inf)


def bf16_rounding_margin(x):
    """Relative distance of x to the nearest bfloat16 rounding boundary: a
    value computed with relative error below this margin rounds to the same
    bfloat16 as x itself."""
    return _rounding_margin(x, 8, -126)


def e4m3_rounding_margin(x):
    """Relative distance of x to the nearest E4M3FN rounding boundary below
    the saturation value 448 (above it every value saturates to 448)."""
    x = np.asarray(x, np.float64)
    return np.where(np.abs(x) >= 448.0, np.inf, _rounding_margin(x, 4, -6))
