"""Pins of the oracle's blocking and statistics against textbook definitions.

Sec. 3 / Sec. 5.B: min, max, and the zero-mean standard deviation of each
block. The exactly rounded sum of squares is pinned to exact rational
arithmetic (fractions.Fraction), independent of the oracle's Dekker split.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import blocks as bk
from oracle.exactsum import exact_squares, sum_of_squares


def _exact_sumsq(x):
    return float(sum(Fraction(float(v)) ** 2 for v in np.ravel(x)))


@pytest.mark.parametrize("seed", range(5))
def test_sum_of_squares_is_exactly_rounded(seed):
    r = np.random.default_rng(seed)
    # wide dynamic range so that naive summation orders disagree
    x = r.standard_normal(300) * np.exp2(r.integers(-30, 30, 300))
    assert sum_of_squares(x) == _exact_sumsq(x)


def test_sum_of_squares_absorption_case():
    # one large square followed by many small ones: any left-to-right or
    # blocked summation that meets the large value first drops the small ones
    x = np.array([2.0 ** 30] + [1.0] * 1000)
    assert sum_of_squares(x) == _exact_sumsq(x) == 2.0 ** 60 + 1024.0


def test_exact_squares_error_free():
    r = np.random.default_rng(3)
    x = r.standard_normal(200) * 1e3
    hi, lo = exact_squares(x)
    for v, h, l in zip(x, hi, lo):
        assert Fraction(float(h)) + Fraction(float(l)) == Fraction(float(v)) ** 2


def test_block_stats_definitions():
    r = np.random.default_rng(7)
    X = r.standard_normal((130, 70))
    L = 64
    st = bk.all_block_stats(X, L)
    assert len(st) == 3 and len(st[0]) == 2
    for i in range(3):
        for j in range(2):
            sub = X[i * L:(i + 1) * L, j * L:(j + 1) * L]
            s = st[i][j]
            assert s.n == sub.size                      # valid elements only
            assert s.mn == min(sub.ravel().tolist())
            assert s.mx == max(sub.ravel().tolist())
            assert s.amax == max(abs(s.mn), s.mx)
            assert s.sumsq == _exact_sumsq(sub)
            assert s.sigma == math.sqrt(_exact_sumsq(sub) / sub.size)
    # a border block: 130 = 2*64 + 2 rows, 70 = 64 + 6 columns
    assert st[2][1].n == 2 * 6


def test_block_zero_fill_and_extent():
    X = np.arange(1, 1 + 5 * 7, dtype=float).reshape(5, 7)
    b = bk.block(X, 1, 1, 4)
    assert b.shape == (4, 4)
    np.testing.assert_array_equal(b[:1, :3], X[4:5, 4:7])
    assert np.all(b[1:, :] == 0) and np.all(b[:, 3:] == 0)
    assert bk.valid_extent(7, 1, 4) == 3 and bk.valid_extent(8, 1, 4) == 4
    assert bk.n_blocks(7, 4) == 2 and bk.n_blocks(8, 4) == 2 and bk.n_blocks(9, 4) == 3


def test_negative_only_block_amax():
    X = -np.abs(np.random.default_rng(1).standard_normal((8, 8))) - 1.0
    s = bk.block_stats(X, 0, 0, 8)
    assert s.mx < 0 and s.amax == -s.mn
