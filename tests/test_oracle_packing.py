"""Pins of the oracle's companding, packing, packed products and unpacking.

What pins them (none of it re-runs the oracle's own formulas):

* eq. (8) expanded in exact rational arithmetic: the packed words equal
  sum_i z^i q_i exactly, and abar . bbar equals the wanted inner product
  plus the W^2 - W side outputs z^(i-h) q_a,i q_b,h;
* brute-force int64 products: inside the exact regime (Prop. 1 with the
  rounding-error bound) the unpacked integers equal them, for both forms;
* hand-built packed values whose unpacking is known by construction;
* Prop. 1 numbers computed by hand (eqs. 15-17) and Remark 2's storage sizes.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import packing as pk


def _ints(rng, shape, q):
    return rng.integers(-q, q + 1, shape).astype(np.float64)


@pytest.mark.parametrize("W", [2, 3, 4])
def test_packed_words_and_eq8_expansion_exact(W):
    rng = np.random.default_rng(100 + W)
    L, q, p = 12, 9, 8                       # small enough to be exact in FP64
    qa = _ints(rng, (L, L), q)
    qb = _ints(rng, (L, L), q)
    abar = pk.pack_sym_a(qa, W, p, "f64")
    bbar = pk.pack_sym_b(qb, W, p, "f64")
    z = Fraction(1, 2 ** p)
    assert abar.shape == (L, L // W) and bbar.shape == (L // W, L)
    for m in range(L):
        for nb in range(L // W):
            want = sum(z ** i * Fraction(qa[m, W * nb + i]) for i in range(W))
            assert Fraction(abar[m, nb]) == want
    for mb in range(L // W):
        for n in range(L):
            want = sum(z ** -i * Fraction(qb[W * mb + i, n]) for i in range(W))
            assert Fraction(bbar[mb, n]) == want
    # eq. (8): the exact product = wanted output + side outputs o_ih = z^(i-h) qa qb
    for (m, n) in [(0, 0), (3, 7), (L - 1, L - 1)]:
        lhs = sum(Fraction(abar[m, j]) * Fraction(bbar[j, n]) for j in range(L // W))
        wanted = sum(Fraction(qa[m, k]) * Fraction(qb[k, n]) for k in range(L))
        side = sum(z ** (i - h) * Fraction(qa[m, W * j + i]) * Fraction(qb[W * j + h, n])
                   for j in range(L // W) for i in range(W) for h in range(W) if i != h)
        assert lhs == wanted + side


@pytest.mark.parametrize("W", [2, 3, 4])
def test_asym_packed_words_exact(W):
    rng = np.random.default_rng(7 + W)
    L, q, p = 12, 5, 6
    qa = _ints(rng, (L, L), q)
    abar = pk.pack_asym_a(qa, W, p, "f64")
    assert abar.shape == (L // W, L)
    z = Fraction(1, 2 ** p)
    for mb in range(L // W):
        for n in range(L):
            assert Fraction(abar[mb, n]) == sum(z ** i * Fraction(qa[W * mb + i, n]) for i in range(W))


def _sym_roundtrip(qa, qb, W, p, prec):
    rbar = pk.packed_product(pk.pack_sym_a(qa, W, p, prec), pk.pack_sym_b(qb, W, p, prec), prec)
    return pk.unpack_sym(rbar, p, prec)


def _asym_roundtrip(qa, qb, W, p, prec):
    rbar = pk.packed_product(pk.pack_asym_a(qa, W, p, prec), qb.astype(pk.DTYPES[prec]), prec)
    return pk.unpack_asym(rbar, W, p, prec)


# q is the largest range inside the exact regime for each case (the most
# demanding point of the predicate), plus smaller ranges.
@pytest.mark.parametrize("form,prec,W,L,q", [
    ("sym", "f64", 2, 64, 295), ("sym", "f64", 2, 64, 100), ("sym", "f64", 4, 64, 5),
    ("sym", "f64", 2, 128, 181), ("sym", "f32", 2, 64, 1), ("sym", "f32", 2, 16, 5),
    ("sym", "f64", 3, 48, 26), ("asym", "f64", 2, 64, 161), ("asym", "f64", 2, 64, 50),
    ("asym", "f64", 4, 64, 3), ("asym", "f64", 2, 128, 104), ("asym", "f32", 2, 64, 1),
    ("asym", "f64", 3, 48, 15), ("sym", "f64", 3, 96, 15), ("sym", "f64", 2, 96, 209),
    ("asym", "f64", 3, 96, 8), ("asym", "f64", 2, 96, 126)])
def test_unpack_equals_bruteforce_in_exact_regime(form, prec, W, L, q):
    rng = np.random.default_rng(L * 1000 + q + W)
    qa = _ints(rng, (L, L), q).astype(pk.DTYPES[prec])
    qb = _ints(rng, (L, L), q).astype(pk.DTYPES[prec])
    r_safe = float(L) * q * q
    p = pk.packing_exponent(r_safe)
    n = L // W if form == "sym" else L
    pred = (pk.exact_regime_sym if form == "sym" else pk.exact_regime_asym)(n, q, q, W, p, r_safe, prec)
    assert pred, "case chosen inside the exact regime"
    r = (_sym_roundtrip if form == "sym" else _asym_roundtrip)(qa, qb, W, p, prec)
    exact = qa.astype(np.int64) @ qb.astype(np.int64)
    np.testing.assert_array_equal(r.astype(np.int64), exact)


def test_errors_appear_beyond_capacity():
    """Sec. 4.A: past the error-free limit the unpacked results gradually pick up
    representation errors (FP32, W = 2, large R)."""
    rng = np.random.default_rng(5)
    L, q = 64, 60
    qa = _ints(rng, (L, L), q).astype(np.float32)
    qb = _ints(rng, (L, L), q).astype(np.float32)
    p = pk.packing_exponent(float(L) * q * q)
    assert not pk.exact_regime_sym(L // 2, q, q, 2, p, float(L) * q * q, "f32")
    r = _sym_roundtrip(qa, qb, 2, p, "f32")
    exact = qa.astype(np.int64) @ qb.astype(np.int64)
    err = r.astype(np.float64) - exact
    assert np.any(err != 0)
    assert np.sqrt(np.mean(err ** 2)) < 0.01 * float(L) * q * q   # gradual, not catastrophic


def test_unpack_sym_handbuilt():
    p = 10
    for wanted, upper, lower in [(5, 3, 0.2), (-7, -2, -0.3), (0, 11, 0.49), (300, -1, 0.0)]:
        rbar = np.array([[upper * 2.0 ** p + wanted + lower]])
        assert pk.unpack_sym(rbar, p, "f64")[0, 0] == wanted


def test_unpack_asym_handbuilt():
    p, W = 9, 3
    z = 2.0 ** -p
    r0, r1, r2 = 17.0, -5.0, 33.0
    rbar = np.array([[r0 + z * r1 + z * z * r2]])
    out = pk.unpack_asym(rbar, W, p, "f64")
    assert out.shape == (3, 1)
    assert list(out[:, 0]) == [r0, r1, r2]


def test_compand_round_half_even():
    x = np.array([0.5, 1.5, 2.5, -0.5, -1.5, 0.49999999999999994, 3.2])
    np.testing.assert_array_equal(pk.compand(x, 1.0, "f64"), [0, 2, 2, -0, -2, 0, 3])
    np.testing.assert_array_equal(pk.compand(np.array([0.3]), 10.0, "f64"), [3.0])


def test_prop1_numbers_by_hand():
    # eq. (17): R_max for c = 1, L = 288, max|A| = 22, max|B| = 1 (Sec. 4.B) is 6336
    assert pk.rmax_eq17(1.0, 1.0, 288, 22.0, 1.0) == 6336.0
    assert pk.rmax_eq17(1.0, 1.0, 288, 22.0, 63.0) == 399168.0
    # eq. (15): z <= 1 / (2 R + u_safe)
    assert pk.z_bound_eq15(6336.0) == 1.0 / 12722.0
    # p: smallest integer with 2^p >= 2R + 50
    for R in [0.0, 1.0, 7.0, 6336.0, 2.0 ** 20, 2.0 ** 20 - 25.0]:
        v = 2 * R + 50
        want = 0
        while 2.0 ** want < v:
            want += 1
        assert pk.packing_exponent(R) == want
    # eq. (16) with u_sys = 2^-52: W_ef = 3 at R = 6336 and R = 82000, 2 at R = 83000
    for R, want in [(6336.0, 3), (82000.0, 3), (83000.0, 2)]:
        z = 1.0 / (2 * R + 50)
        assert pk.w_ef_eq16(R, z, 2.0 ** -52) == want
    # by hand: (ln 12673 - 52 ln 2) / (-ln 12722) + 1 = (9.44724 - 36.04365) / (-9.45109) + 1 = 3.8141
    assert abs(math.log(12673 * 2.0 ** -52) / math.log(1 / 12722) + 1 - 3.8141) < 1e-3


@pytest.mark.parametrize("W,L", [(2, 64), (4, 64), (3, 96), (2, 96)])
def test_remark2_storage(W, L):
    """Remark 2: symmetric packing stores 2 L^2 / W words, asymmetric L^2 (1 + 1/W)."""
    qa = np.zeros((L, L))
    sym_words = pk.pack_sym_a(qa, W, 10, "f64").size + pk.pack_sym_b(qa, W, 10, "f64").size
    asym_words = pk.pack_asym_a(qa, W, 10, "f64").size + qa.size
    assert sym_words == 2 * L * L // W
    assert asym_words == L * L + L * L // W


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_lsum_is_one_fused_multiply_add_per_pair(prec):
    """Eqs. (5) and (2): C = fma(r, 1/(c_A c_B), C) for l ascending from 0, one
    rounding per pair in the packing precision (W = 1 pairs add their native
    product) -- checked against exact rational arithmetic on sampled outputs,
    on a case where multiply-then-add would round differently somewhere."""
    from fractions import Fraction

    from oracle import pipeline as pl
    from tests.oracle_tables import tables
    from tests.test_oracle_precision import _round_f32
    rng = np.random.default_rng(5 if prec == "f64" else 6)
    L, nl = 64, 5
    A = rng.standard_normal((L, nl * L)) * rng.uniform(0.5, 4.0, (1, nl * L))
    B = rng.laplace(0.0, 1.0, (nl * L, L))
    if prec == "f32":
        A, B = A.astype(np.float32), B.astype(np.float32)
    cfg = pl.Config(L=L, form="sym", prec=prec, ctrl="snr", snr_db=30.0 if prec == "f64" else 12.0,
                    w_allowed=(1, 2))
    res = pl.run(A, B, cfg, calib=tables(L, "sym", prec, (2,)), keep=True)
    rnd = (lambda x: float(x)) if prec == "f64" else _round_f32
    dt = np.float64 if prec == "f64" else np.float32
    ws = [res.plan.chosen[(0, 0, l)].W for l in range(nl)]
    assert 2 in ws
    differs = 0
    for (m, n) in [(int(a), int(b)) for a, b in rng.integers(0, L, (60, 2))]:
        acc, naive = Fraction(0), dt(0.0)
        for l in range(nl):
            o = res.plan.chosen[(0, 0, l)]
            r = res.traces[(0, 0, l)].r[m, n]
            inv = 1.0 if o.W == 1 else float(dt(o.inv))
            acc = Fraction(rnd(Fraction(float(r)) * Fraction(inv) + acc))
            naive = naive + (dt(r) if o.W == 1 else dt(r) * dt(o.inv))
        assert res.C[m, n] == dt(float(acc)), (m, n)
        differs += int(dt(float(acc)) != naive)
    assert differs > 0
