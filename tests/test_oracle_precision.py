"""Pins of the INT8 / FP8 block-scaled oracle (oracle/precision.py)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import blocks as bk
from oracle import noise as nz
from oracle import precision as pr

FINITE = [c for c in range(256) if (c & 0x7F) != 0x7F]


def test_e4m3_code_table():
    """OCP E4M3FN: bias 7, 3 mantissa bits, subnormal step 2^-9, max 448, NaN S.1111.111."""
    assert pr.e4m3_decode(0x00) == 0.0 and math.copysign(1, pr.e4m3_decode(0x80)) < 0
    assert pr.e4m3_decode(0x01) == 2.0 ** -9
    assert pr.e4m3_decode(0x07) == 7 * 2.0 ** -9
    assert pr.e4m3_decode(0x08) == 2.0 ** -6          # smallest normal
    assert pr.e4m3_decode(0x38) == 1.0
    assert pr.e4m3_decode(0x3C) == 1.5
    assert pr.e4m3_decode(0x7E) == 448.0              # largest finite
    assert pr.e4m3_decode(0xFE) == -448.0
    assert math.isnan(pr.e4m3_decode(0x7F)) and math.isnan(pr.e4m3_decode(0xFF))
    pos = sorted(pr.e4m3_decode(c) for c in range(1, 0x7F))
    assert len(set(pos)) == 126 and all(a < b for a, b in zip(pos, pos[1:]))


def test_e4m3_round_trip():
    for c in FINITE:
        v = pr.e4m3_decode(c)
        assert pr.e4m3_round(v) == v
        assert pr.e4m3_encode(v) == c


def _nearest_brute(v):
    vals = sorted({pr.e4m3_decode(c) for c in FINITE})
    best = min(abs(v - x) for x in vals)
    cands = [x for x in vals if abs(v - x) == best]
    if len(cands) == 1:
        return cands[0]
    even = [x for x in cands if (pr.e4m3_encode(x) & 1) == 0]   # tie: even mantissa
    assert len(even) == 1
    return even[0]


def test_e4m3_round_nearest_even_brute_force():
    vals = sorted({pr.e4m3_decode(c) for c in FINITE})
    mids = [(a + b) / 2 for a, b in zip(vals, vals[1:])]        # every tie
    rng = np.random.default_rng(5)
    probe = mids + list(rng.uniform(-448, 448, 400)) + list(rng.uniform(-0.05, 0.05, 200))
    for v in probe:
        assert pr.e4m3_round(v) == _nearest_brute(v), v


def test_e4m3_saturates():
    assert pr.e4m3_round(448.0 * (1 + 2 ** -40)) == 448.0
    assert pr.e4m3_round(463.9) == 448.0
    assert pr.e4m3_round(1e6) == 448.0 and pr.e4m3_round(-1e6) == -448.0


def test_integer_blocks_at_full_range_are_exact():
    """max|X| = Q in every block makes every scale 1: the form is the exact
    integer product (textbook matmul)."""
    rng = np.random.default_rng(3)
    L, Q = 64, 127
    A = rng.integers(-Q, Q + 1, (128, 192)).astype(np.float64)
    B = rng.integers(-Q, Q + 1, (192, 64)).astype(np.float64)
    for X in (A, B):
        for r in range(0, X.shape[0], L):
            for c in range(0, X.shape[1], L):
                X[r, c] = Q
    res = pr.run(A, B, L, "i8", float(Q))
    exact = A.astype(np.int64) @ B.astype(np.int64)
    assert np.array_equal(res.C.astype(np.int64), exact)
    assert np.all(res.scale_a == 1.0) and np.all(res.scale_b == 1.0)


def test_int8_products_are_bruteforce_integer_products():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((100, 150))
    B = rng.laplace(0, 1, (150, 70))
    res = pr.run(A, B, 64, "i8", 127.0)
    for (i, j, l), r in list(res.products.items())[:6]:
        a = res.qa[i * 64:(i + 1) * 64, l * 64:(l + 1) * 64].astype(np.int64)
        b = res.qb[l * 64:(l + 1) * 64, j * 64:(j + 1) * 64].astype(np.int64)
        brute = np.array([[sum(int(a[m, k]) * int(b[k, n]) for k in range(64)) for n in range(3)]
                          for m in range(3)])
        assert np.array_equal(r[:3, :3], brute)
    assert np.max(np.abs(res.qa)) <= 127 and np.max(np.abs(res.qb)) <= 127


@pytest.mark.parametrize("dist", ["gaussian", "laplace"])
def test_int8_snr_matches_prop2(dist):
    """Uniform rounding at c = Q / max|X|: the measured output SNR matches eqs.
    19-20 evaluated per pair (Prop. 2), within 0.5 dB."""
    rng = np.random.default_rng(9)
    L, n = 128, 384
    draw = rng.standard_normal if dist == "gaussian" else (lambda s: rng.laplace(0, 1, s))
    A, B = draw((n, n)), draw((n, n))
    res = pr.run(A, B, L, "i8", 127.0, keep_products=False)
    exact = A @ B
    snr = 10 * math.log10(float(np.sum(exact ** 2)) / float(np.sum((res.C - exact) ** 2)))
    sig = noise = 0.0
    nb = n // L
    for i in range(nb):
        for j in range(nb):
            for l in range(nb):
                sa, sb = res.stats_a[i][l], res.stats_b[l][j]
                ca, cb = res.scale_a[i, l], res.scale_b[l, j]
                sig += L * sa.sigma ** 2 * sb.sigma ** 2
                noise += nz.quant_noise_eq19(L, sa.sigma, sb.sigma, ca, cb)
    pred = 10 * math.log10(sig / noise)
    assert abs(snr - pred) < 0.5, (snr, pred)


def test_fp8_rounding_bound_and_grid():
    rng = np.random.default_rng(11)
    A = rng.laplace(0, 1, (128, 128))
    B = rng.standard_normal((128, 128))
    res = pr.run(A, B, 128, "e4m3", 448.0)
    v = A * res.scale_a[0, 0]
    q = res.qa[:128, :128]
    normal = np.abs(v) >= 2.0 ** -6
    assert np.all(np.abs(q - v)[normal] <= 2.0 ** -4 * np.abs(v)[normal])   # half a 3-bit ulp
    assert np.all(np.abs(q - v)[~normal] <= 2.0 ** -10)
    assert np.max(np.abs(q)) == 448.0
    codes = pr.codes(q, "e4m3")
    assert all(pr.e4m3_decode(int(c)) == x for c, x in zip(codes.ravel()[:500], q.ravel()[:500]))
    assert pr.exact_fp8_sums_fit(128)


def _round_f32(x: Fraction) -> float:
    """The float32 value nearest to the rational x (ties to even), exactly."""
    if x == 0:
        return 0.0
    sign = -1 if x < 0 else 1
    x = abs(x)
    e = x.numerator.bit_length() - x.denominator.bit_length()   # 2^(e-1) <= x < 2^(e+1)
    while x >= Fraction(2) ** (e + 1):
        e += 1
    while x < Fraction(2) ** e:
        e -= 1
    q = max(e, -126) - 23                                  # ulp of the binade (subnormals below 2^-126)
    m = x / Fraction(2) ** q
    n, r = divmod(m.numerator, m.denominator)
    if 2 * r > m.denominator or (2 * r == m.denominator and n % 2 == 1):
        n += 1
    return sign * float(Fraction(n) * Fraction(2) ** q)


def test_epilogue_is_one_fused_multiply_add_per_pair():
    """Reverse companding and the l-sum: C = fma(float32(r), float32(1/(c_A c_B)), C)
    for l ascending from 0, each step rounded once to float32 -- checked against
    exact rational arithmetic, on outputs where multiply-then-add rounds differently."""
    rng = np.random.default_rng(21)
    L = 64
    A = rng.laplace(0, 1, (L, 4 * L)) * rng.uniform(0.5, 3.0, (1, 4 * L))
    B = rng.standard_normal((4 * L, L))
    res = pr.run(A, B, L, "i8", 127.0)
    invs = [np.float32(res.options[(0, 0, l)].inv) for l in range(4)]
    differs = 0
    for (m, n) in [(int(a), int(b)) for a, b in rng.integers(0, L, (40, 2))]:
        acc, naive = 0.0, np.float32(0.0)
        for l in range(4):
            r = int(res.products[(0, 0, l)][m, n])
            acc = _round_f32(Fraction(r) * Fraction(float(invs[l])) + Fraction(acc))
            naive = naive + np.float32(r) * invs[l]
        assert res.C[m, n] == np.float32(acc), (m, n)
        differs += int(np.float32(acc) != naive)
    assert differs > 0        # the sample tells the two readings apart
