"""The plan kernel's pruning by ranks and bisection equals the Sec. 6 greedy.

When every pair's D falls strictly along its allowed W (weakly to the W = 1
floor), the plan kernel does not run the greedy one removal at a time: it
ranks all entries (pair l at level v with D > 0) by descending D, lowest l
first among equals, and finds the greedy's stopping point by bisection over
that ranking -- the first cut whose exactly rounded sum is within the budget
(SNR control), or, when no drop adds saved work, the last cut that keeps the
saving at the target (throughput control); unavailable options rank first and
always go. This file restates that procedure on the host and checks it
against the oracle's greedy (``prune``, ``prune_accel``) on small inner kernels
with ties, zero entries, unavailable options and budgets that sit exactly on
a partial sum. The GPU tests check the kernel against the same greedy.
"""
import pytest
from hypothesis import given, settings, strategies as st

from oracle import control as ct
from oracle.exactsum import exact_sum


def _opt(W, d):
    return ct.PairOption(W=W, r_max=0.0, c_a=1.0, c_b=1.0, q_a=0.0, q_b=0.0, r_safe=0.0, p=0,
                         inv=1.0, d=d, nsr=0.0, s_rep=0.0)


def _monotone(options, w_desc):
    n_ent = len(w_desc) - 1
    for opt in options:
        for v in range(n_ent):
            d0, d1 = opt[w_desc[v]].d, opt[w_desc[v + 1]].d
            if not d1 <= d0:
                return False
            if v + 1 < n_ent and d1 > 0.0 and not d0 > d1:
                return False
    return True


def _ranking(options, w_desc):
    """Entries (D, l, v) with D > 0: larger D first, lower l first among equals."""
    ent = [(opt[w_desc[v]].d, l, v) for l, opt in enumerate(options) for v in range(len(w_desc) - 1)
           if opt[w_desc[v]].d > 0.0]
    ent.sort(key=lambda e: (-e[0], e[1]))
    return ent


def _levels(options, ent, cut):
    level = [0] * len(options)
    for _, l, _ in ent[:cut]:
        level[l] += 1
    return level


def prune_by_rank(options, w_desc, d_kernel):
    ent = _ranking(options, w_desc)
    n_pos = len(ent)
    n_unav = sum(1 for e in ent if e[0] >= ct.D_UNAVAILABLE)

    def total(cut):
        lv = _levels(options, ent, cut)
        return exact_sum(options[l][w_desc[lv[l]]].d for l in range(len(options)))

    def within(x):                     # the greedy's stopping test
        return not x > d_kernel

    if not within(total(n_pos)):
        level = [len(w_desc) - 1] * len(options)
    else:
        lo, hi = n_unav, n_pos
        while lo < hi:
            mid = (lo + hi) // 2
            if within(total(mid)):
                hi = mid
            else:
                lo = mid + 1
        level = _levels(options, ent, lo)
    return [w_desc[v] for v in level]


def prune_accel_by_rank(options, w_desc, frac, units=None):
    ent = _ranking(options, w_desc)
    n_pos = len(ent)
    n_unav = sum(1 for e in ent if e[0] >= ct.D_UNAVAILABLE)
    nl = len(options)
    own = nl * ct.saved_units(w_desc[0], units)
    target = ct.accel_target(nl, w_desc[0], frac, units)
    delta = [ct.saved_units(w_desc[v], units) - ct.saved_units(w_desc[v + 1], units)
             for v in range(len(w_desc) - 1)]
    assert all(x >= 0 for x in delta)

    def saved(cut):
        return own - sum(delta[v] for _, _, v in ent[:cut])

    lo, hi = n_unav, n_pos
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if not float(saved(mid)) < target:
            lo = mid
        else:
            hi = mid - 1
    return [w_desc[v] for v in _levels(options, ent, lo)]


W_SETS = [(2, 1), (4, 2, 1), (3, 2, 1), (4, 3, 2, 1)]
D_GRID = [0.25, 0.5, 1.0, 1.5, 2.0, 3.0]     # few values, so that equal D across pairs is common


@st.composite
def inner_kernel(draw):
    w_desc = list(draw(st.sampled_from(W_SETS)))
    nl = draw(st.integers(1, 10))
    options = []
    for _ in range(nl):
        # strictly falling D along the entry levels, then possibly zeros, W = 1 at 0
        n_ent = len(w_desc) - 1
        ds = sorted(draw(st.lists(st.sampled_from(D_GRID), min_size=n_ent, max_size=n_ent, unique=True)),
                    reverse=True)
        nz = draw(st.integers(0, n_ent))          # trailing entries with D = 0
        ds = ds[:n_ent - nz] + [0.0] * nz
        if draw(st.integers(0, 5)) == 0 and ds[0] > 0.0:
            ds[0] = ct.D_UNAVAILABLE               # an option the table cannot supply
        opt = {W: _opt(W, d) for W, d in zip(w_desc[:-1], ds)}
        opt[1] = _opt(1, 0.0)
        options.append(opt)
    return w_desc, options


@settings(max_examples=400, deadline=None)
@given(inner_kernel(), st.integers(0, 40), st.sampled_from([0.0, 1.0, -1.0]))
def test_snr_prune_by_rank_equals_greedy(kern, k, shift):
    """Budgets on an exact partial sum, just below it and just above it."""
    w_desc, options = kern
    assert _monotone(options, w_desc)
    ent = _ranking(options, w_desc)
    cut = min(k, len(ent))
    lv = _levels(options, ent, cut)
    b = exact_sum(options[l][w_desc[lv[l]]].d for l in range(len(options)))
    if shift:
        b = b * (1.0 + shift * 2.0 ** -52) if b > 0.0 else (2.0 ** -1074 if shift > 0 else 0.0)
    assert prune_by_rank(options, w_desc, b) == ct.prune(options, w_desc, b)


@settings(max_examples=100, deadline=None)
@given(inner_kernel())
def test_nan_budget_and_target_stop_like_the_greedy(kern):
    """A NaN budget stops the greedy at once (after the unavailable options), and
    a NaN throughput target never stops it: the bisections take the greedy's own
    comparisons, so they agree there too."""
    w_desc, options = kern
    nan = float("nan")
    assert prune_by_rank(options, w_desc, nan) == ct.prune(options, w_desc, nan)
    assert prune_accel_by_rank(options, w_desc, nan) == ct.prune_accel(options, w_desc, nan)


@settings(max_examples=400, deadline=None)
@given(inner_kernel(), st.sampled_from([0.0, 0.1, 0.25, 1 / 3, 0.5, 0.6, 0.75, 0.9, 1.0]),
       st.sampled_from([None, {2: 1365, 3: 1800, 4: 2365}, {2: 2048, 3: 2048, 4: 3072}]))
def test_accel_prune_by_rank_equals_greedy(kern, frac, units):
    """Nominal twelfths and measured units in which no drop adds saved work
    (equal units for two packings make some drops save nothing)."""
    w_desc, options = kern
    assert prune_accel_by_rank(options, w_desc, frac, units) == ct.prune_accel(options, w_desc, frac, units)


def test_gaining_units_are_left_to_the_greedy():
    """With measured units in which a smaller W saves more, dropping a pair
    adds saved work, the saving is no longer monotone along the ranking, and the
    kernel runs the greedy step by step: the bisection's precondition fails."""
    units = {2: 1365, 4: 900}
    w_desc = [4, 2, 1]
    delta = [ct.saved_units(w_desc[v], units) - ct.saved_units(w_desc[v + 1], units) for v in range(2)]
    assert min(delta) < 0
    with pytest.raises(AssertionError):
        prune_accel_by_rank([{4: _opt(4, 2.0), 2: _opt(2, 1.0), 1: _opt(1, 0.0)}], w_desc, 0.5, units)
