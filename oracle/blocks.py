"""Inner-kernel blocking and per-block statistics (oracle; test infrastructure only).

Sec. 2, eqs. (1)-(2): C = A B is split into L x L inner kernels
R_ij = sum_l A_il B_lj. Matrices whose sizes are not multiples of L get
"cleanup" handling at the borders, which the paper omits; the reading taken
here is zero fill: out-of-range elements of a border block are 0, block
statistics cover the valid elements only, and a pair's inner extent L_eff is
the number of valid columns of A_il (= valid rows of B_lj).

Sec. 3 and Sec. 5.B: for every block the method needs min, max and the
standard deviation. Inputs are modelled as zero-mean, so sigma is read as the
root mean square sqrt(sum x^2 / n) over the n valid elements -- the quantity
the signal power L sigma_a^2 sigma_b^2 of eq. (20) uses.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .exactsum import sum_of_squares


def n_blocks(extent: int, L: int) -> int:
    """Number of L-blocks covering an extent (ceil division)."""
    return (extent + L - 1) // L


def block(X: np.ndarray, r: int, c: int, L: int) -> np.ndarray:
    """Block (r, c) of X as an L x L float array, zero-filled past the borders."""
    out = np.zeros((L, L), dtype=X.dtype)
    sub = X[r * L:(r + 1) * L, c * L:(c + 1) * L]
    out[:sub.shape[0], :sub.shape[1]] = sub
    return out


def valid_extent(extent: int, b: int, L: int) -> int:
    """Valid length of block index b along an axis of the given extent."""
    return min(L, extent - b * L)


@dataclass(frozen=True)
class BlockStats:
    """Statistics of one block over its valid elements (Sec. 3, Sec. 5.B)."""
    mn: float        # min{X}
    mx: float        # max{X}
    sumsq: float     # exactly rounded sum of squares
    n: int           # number of valid elements

    @property
    def amax(self) -> float:
        """max{|min{X}|, max{X}}, the range bound of eq. (17)."""
        return max(abs(self.mn), self.mx)

    @property
    def sigma(self) -> float:
        """RMS sqrt(sumsq / n): the zero-mean standard deviation."""
        return math.sqrt(self.sumsq / self.n)


def block_stats(X: np.ndarray, r: int, c: int, L: int) -> BlockStats:
    """Stats of block (r, c) of X (valid elements only)."""
    sub = np.asarray(X[r * L:(r + 1) * L, c * L:(c + 1) * L], dtype=np.float64)
    return BlockStats(float(sub.min()), float(sub.max()), sum_of_squares(sub), int(sub.size))


def all_block_stats(X: np.ndarray, L: int) -> list[list[BlockStats]]:
    """Stats of every block of X, indexed [row-block][col-block]."""
    R, C = n_blocks(X.shape[0], L), n_blocks(X.shape[1], L)
    return [[block_stats(X, r, c, L) for c in range(C)] for r in range(R)]
