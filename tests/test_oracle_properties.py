"""Property-based pins of the oracle on random tiny cases (hypothesis).

* Packing (eqs. 6-14): for random small shapes, ranges and W, whenever the
  exact-regime predicate (Prop. 1 with the rounding-error bound) holds, the
  unpacked integers equal the brute-force int64 product, in both forms and both
  packing precisions.
* Pruning (Sec. 6): the greedy removal sequence does not depend on the budget,
  only where it stops. So a looser distortion budget never gives a subblock a
  smaller W, and a smaller throughput fraction never gives a larger one. After
  distortion pruning, the budget is met unless every subblock is at the
  smallest allowed W.
"""
from types import SimpleNamespace

import numpy as np
import pytest

from oracle import control as ct
from oracle import packing as pk

hyp = pytest.importorskip("hypothesis")
from hypothesis import assume, given, settings  # noqa: E402
from hypothesis import strategies as st  # noqa: E402


@settings(max_examples=150, deadline=None)
@given(form=st.sampled_from(["sym", "asym"]), prec=st.sampled_from(["f64", "f32"]),
       W=st.integers(2, 4), rows=st.integers(1, 3), cols=st.integers(1, 5), inner=st.integers(1, 6),
       qbits=st.integers(0, 14), seed=st.integers(0, 2 ** 31 - 1))
def test_packing_exact_in_regime(form, prec, W, rows, cols, inner, qbits, seed):
    m = rows * W if form == "asym" else rows
    k = inner * W if form == "sym" else inner
    q = (1 << qbits) - 1 if qbits else 1
    r_safe = float(k) * q * q
    p = pk.packing_exponent(r_safe)
    n = k // W if form == "sym" else k
    pred = (pk.exact_regime_sym if form == "sym" else pk.exact_regime_asym)(n, q, q, W, p, r_safe, prec)
    assume(pred)
    rng = np.random.default_rng(seed)
    dt = pk.DTYPES[prec]
    qa = rng.integers(-q, q + 1, (m, k)).astype(dt)
    qb = rng.integers(-q, q + 1, (k, cols)).astype(dt)
    if form == "sym":
        rbar = pk.packed_product(pk.pack_sym_a(qa, W, p, prec), pk.pack_sym_b(qb, W, p, prec), prec)
        r = pk.unpack_sym(rbar, p, prec)
    else:
        rbar = pk.packed_product(pk.pack_asym_a(qa, W, p, prec), qb, prec)
        r = pk.unpack_asym(rbar, W, p, prec)
    exact = qa.astype(np.int64) @ qb.astype(np.int64)
    np.testing.assert_array_equal(np.asarray(r).astype(np.int64), exact)


def _options(ds, w_desc):
    return [{w: SimpleNamespace(d=float(dl[i])) for i, w in enumerate(w_desc)} for dl in ds]


_W_SETS = [[4, 2, 1], [2, 1], [3, 2, 1], [4, 1]]


@st.composite
def _pairs(draw):
    w_desc = draw(st.sampled_from(_W_SETS))
    nl = draw(st.integers(1, 12))
    ds = []
    for _ in range(nl):
        row = [draw(st.floats(0.0, 1e3, allow_nan=False)) for _ in w_desc[:-1]]
        ds.append(row + [0.0])                 # W = 1 adds no noise
    return w_desc, ds


@settings(max_examples=200, deadline=None)
@given(case=_pairs(), b1=st.floats(0.0, 5e3), b2=st.floats(0.0, 5e3))
def test_prune_monotone_in_budget(case, b1, b2):
    w_desc, ds = case
    lo, hi = min(b1, b2), max(b1, b2)
    opts = _options(ds, w_desc)
    w_lo = ct.prune(opts, w_desc, lo)
    w_hi = ct.prune(opts, w_desc, hi)
    assert all(a >= b for a, b in zip(w_hi, w_lo)), (w_hi, w_lo)
    for wc, bud in ((w_lo, lo), (w_hi, hi)):
        total = sum(opts[l][w].d for l, w in enumerate(wc))
        assert total <= bud * (1 + 1e-12) or all(w == w_desc[-1] for w in wc)


@settings(max_examples=200, deadline=None)
@given(case=_pairs(), f1=st.floats(0.0, 1.0), f2=st.floats(0.0, 1.0))
def test_prune_accel_monotone_in_fraction(case, f1, f2):
    w_desc, ds = case
    lo, hi = min(f1, f2), max(f1, f2)
    opts = _options(ds, w_desc)
    w_lo = ct.prune_accel(opts, w_desc, lo)
    w_hi = ct.prune_accel(opts, w_desc, hi)
    # a larger required fraction of saved work keeps at least as much packing
    assert all(a >= b for a, b in zip(w_hi, w_lo)), (w_hi, w_lo)
    saved = sum(ct.saved_units(w) for w in w_hi)
    assert saved >= ct.accel_target(len(ds), w_desc[0], hi) or w_hi == [w_desc[0]] * len(ds)
