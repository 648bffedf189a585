"""Exactly rounded sums for the oracle (test infrastructure only).

The method needs a handful of sums whose rounding order the paper does not
fix: the block mean square that defines sigma (Sec. 5.B), and the two sums of
the inner-kernel pruning (Sec. 6). The oracle takes the plain definition of a
sum -- the exact real sum, rounded once to the nearest double -- so that the
value does not depend on any summation order. ``math.fsum`` is exactly that.
"""
from __future__ import annotations

import math

import numpy as np

# Veltkamp splitting constant 2^27 + 1 for IEEE binary64.
_SPLIT = 134217729.0


def exact_squares(x: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Return (hi, lo) with hi + lo == x*x exactly, elementwise.

    Dekker's error-free product via Veltkamp splitting (valid for |x| < 2^996);
    hi is the rounded square, lo the exact rounding error.
    """
    x = np.asarray(x, dtype=np.float64).ravel()
    t = _SPLIT * x
    xh = t - (t - x)
    xl = x - xh
    hi = x * x
    lo = ((xh * xh - hi) + 2.0 * xh * xl) + xl * xl
    return hi, lo


def sum_of_squares(x: np.ndarray) -> float:
    """Exactly rounded value of sum(x_i^2) over all elements of x."""
    hi, lo = exact_squares(x)
    return math.fsum(np.concatenate([hi, lo]).tolist())


def exact_sum(values) -> float:
    """Exactly rounded value of the sum of the given doubles."""
    return math.fsum(float(v) for v in values)
