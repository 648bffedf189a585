"""Direct pins of the oracle's calibration measurement (Sec. 4.B, eq. 18) and of
its per-pair option choice (Prop. 4, eq. 27 read as in the noise module), and of
the rule that an option the calibration cannot supply is always pruned (Sec. 6).

Each pin rests on something other than the function it checks:
* measure(): inside the exact regime of Prop. 1 every unpacked integer equals
  the brute-force product, so m = s = 0 exactly; a planted integer error of
  known values added to the packed product gives the eq. (18) mean and RMSE of
  those values (computed here with Python integers); R_max = L max|A| max|B|.
* best_option(): with s = 0 the eq. (27) noise falls strictly with R, so the
  choice is the largest grid R; on a small hand-made table the argmin equals a
  brute force in exact rational arithmetic of the closed form
  L k / (6 R) + L^2 k^2 / (144 R^2) + L k^2 s^2 / R^2 (k = product of the two
  range-to-RMS ratios); equal noise values go to the first (smallest-R) point.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import calibration as cal
from oracle import control as ct
from oracle import packing as pk
from oracle.blocks import BlockStats


def _uniforms(L, inst, seed):
    r = np.random.default_rng(seed)
    return r.random((inst, L, L)), r.random((inst, L, L))


# ---------------------------------------------------------------------------
# measure(): eq. (18)

EXACT_CASES = [  # form, prec, W, L, q: inside Prop. 1's exact regime (checked below)
    ("sym", "f64", 2, 64, 100),
    ("asym", "f64", 2, 64, 100),
    ("asym", "f64", 4, 64, 3),
    ("sym", "f64", 4, 16, 1),
    ("asym", "f64", 3, 96, 6),
    ("sym", "f32", 2, 16, 3),
]


def _exact_regime(form, prec, W, L, q):
    r = float(L * q * q)
    p = pk.packing_exponent(r, 50.0)
    f = pk.exact_regime_sym if form == "sym" else pk.exact_regime_asym
    return f(L, float(q), float(q), W, p, r, prec)


@pytest.mark.parametrize("form,prec,W,L,q", EXACT_CASES)
def test_measure_zero_inside_exact_regime(form, prec, W, L, q):
    """Prop. 1: inside the exact regime the packed path returns the exact integer
    product, so eq. (18) gives m = s = 0 exactly, and R_max = L q^2 (eq. 17, c = 1)."""
    assert _exact_regime(form, prec, W, L, q)
    ua, ub = _uniforms(L, 3, 1000 + L + W)
    r, m, s = cal.measure(L, W, form, prec, q, ua, ub)
    assert r == float(L * q * q)
    assert m == 0.0 and s == 0.0


def test_measure_separate_ranges_r_max():
    """R_max = L max|A| max|B| when the two ranges differ (the paper's protocol)."""
    ua, ub = _uniforms(32, 2, 7)
    r, m, s = cal.measure(32, 2, "sym", "f64", 22, ua, ub, q_b=50)
    assert r == 32.0 * 22.0 * 50.0
    assert m == 0.0 and s == 0.0


def _planted(inst, rows, cols):
    """Known integer errors in {-2, ..., 2} per instance and packed output."""
    x = np.arange(rows)[:, None]
    y = np.arange(cols)[None, :]
    return [((7 * x + 3 * y + 5 * t) % 5 - 2).astype(np.int64) for t in range(inst)]


@pytest.mark.parametrize("form,W", [("sym", 2), ("asym", 2), ("asym", 3), ("asym", 4)])
def test_measure_planted_error(monkeypatch, form, W):
    """A known integer error d added to every packed product word (inside the exact
    regime) reaches the unpacked integers as d: the output of that word (sym) or
    the first row it carries (asym, eq. 14 peels that row first). Eq. (18) must
    give m = sum(d) / n and s = sqrt(sum(d^2) / n) over all n outputs."""
    L, q, inst = 48, 20 if W == 2 else 3, 2
    assert _exact_regime(form, "f64", W, L, q)
    ua, ub = _uniforms(L, inst, 31 + W)
    rows = L if form == "sym" else L // W
    planted = _planted(inst, rows, L)
    calls = {"t": 0}
    orig = pk.packed_product

    def with_error(abar, bbar, prec):
        out = orig(abar, bbar, prec)
        d = planted[calls["t"]]
        calls["t"] += 1
        return out + d.astype(out.dtype)

    monkeypatch.setattr(pk, "packed_product", with_error)
    r, m, s = cal.measure(L, W, form, "f64", q, ua, ub)
    n = inst * L * L
    s1 = sum(int(d.sum()) for d in planted)
    s2 = sum(int((d * d).sum()) for d in planted)
    assert calls["t"] == inst
    assert m == s1 / n
    assert s == math.sqrt(s2 / n)
    assert s > 0.0


def test_measure_mutation_abs_mean_fails(monkeypatch):
    """Planted mistake: the mean error taken over |e|. The planted-error pin fails."""
    monkeypatch.setattr(cal, "exact_sum", lambda v: math.fsum(abs(x) for x in v))
    with pytest.raises(AssertionError):
        test_measure_planted_error(monkeypatch, "sym", 2)


def test_measure_mutation_z_too_large_fails(monkeypatch):
    """Planted mistake: z = 2^-(p-4), four bits too large for eq. (15). The packed
    slots overlap and the exact-regime pin fails."""
    orig = pk.packing_exponent
    monkeypatch.setattr(pk, "packing_exponent", lambda r, u_safe=50.0: orig(r, u_safe) - 4)
    ua, ub = _uniforms(64, 2, 5)
    _, m, s = cal.measure(64, 2, "sym", "f64", 100, ua, ub)
    assert s > 0.0


# ---------------------------------------------------------------------------
# best_option(): Prop. 4 with R* = argmin of the eq. (27) noise

def _stats(rng, n=4096):
    x = rng.standard_normal(n) * rng.uniform(0.5, 3.0)
    x[rng.integers(n)] *= rng.uniform(2.0, 6.0)     # a range-to-RMS ratio away from the bulk
    return BlockStats(float(x.min()), float(x.max()), float(np.sum(x * x)), n)


def _nsr_exact(L, sa, sb, R, s):
    """Closed form of the eq. (27) noise at the eq. (26) companders, exactly:
    L k / (6 R) + L^2 k^2 / (144 R^2) + L k^2 s^2 / R^2 with k = k_A k_B."""
    k = (Fraction(sa.amax) / Fraction(sa.sigma)) * (Fraction(sb.amax) / Fraction(sb.sigma))
    L, R, s = Fraction(L), Fraction(R), Fraction(s)
    return L * k / (6 * R) + L * L * k * k / (144 * R * R) + L * k * k * s * s / (R * R)


@pytest.mark.parametrize("seed", range(6))
def test_best_option_zero_s_takes_largest_r(seed):
    """With s = 0 every term of the noise falls strictly as R grows: R* is the largest R."""
    rng = np.random.default_rng(seed)
    sa, sb = _stats(rng), _stats(rng)
    r = np.array([2.0 ** (10 + 0.25 * k) for k in range(60)])
    o = ct.best_option(2, 64, sa, sb, ct.CalibTable(r, np.zeros_like(r)), 50.0)
    assert o.r_max == r[-1]
    assert o.s_rep == 0.0


def _hand_table():
    r = np.array([2.0 ** k for k in range(12, 30)])
    # zero in the exact regime, then growing faster than R, as a representation error
    # does: the argmin lands inside the grid
    s = np.array([0.0 if k < 16 else 2.0 ** (1.5 * (k - 16)) for k in range(12, 30)])
    s[5] = np.inf                                       # an unusable point is skipped
    return ct.CalibTable(r, s)


@pytest.mark.parametrize("seed", range(8))
def test_best_option_matches_rational_bruteforce(seed):
    """On a hand-made table the chosen R is the exact rational argmin of the closed
    form (compared only where the minimum is unique by a margin well above rounding)."""
    rng = np.random.default_rng(100 + seed)
    sa, sb = _stats(rng), _stats(rng)
    tab = _hand_table()
    L = 64
    vals = [(_nsr_exact(L, sa, sb, R, S), k) for k, (R, S) in enumerate(zip(tab.r, tab.s))
            if math.isfinite(S)]
    vals.sort()
    assert vals[1][0] - vals[0][0] > Fraction(1, 10 ** 9) * vals[0][0]
    o = ct.best_option(2, L, sa, sb, tab, 50.0)
    k = vals[0][1]
    assert o.r_max == tab.r[k] and o.s_rep == tab.s[k]
    assert 0 < k < tab.r.size - 1                       # an interior minimum: s matters


@pytest.mark.parametrize("order", [(0.0, 1e-30), (1e-30, 0.0)])
def test_best_option_tie_goes_to_first(order):
    """Equal noise at two grid points (here the same R with representation terms
    too small to change the rounded noise) goes to the first of them."""
    rng = np.random.default_rng(9)
    sa, sb = _stats(rng), _stats(rng)
    r = np.array([2.0 ** 20, 2.0 ** 40, 2.0 ** 40])
    s = np.array([0.0, order[0], order[1]])
    o = ct.best_option(2, 64, sa, sb, ct.CalibTable(r, s), 50.0)
    assert o.r_max == 2.0 ** 40 and o.s_rep == order[0]


def test_best_option_no_finite_noise_is_unavailable():
    """Blocks whose eq. (27) noise overflows at every grid point get no option (D = 1e300)."""
    big = BlockStats(-1e160, 1e160, 1e300, 4)    # L max|A| max|B| overflows
    r = np.array([2.0 ** 10, 2.0 ** 11])
    o = ct.best_option(2, 64, big, big, ct.CalibTable(r, np.zeros(2)), 50.0)
    assert o.d == ct.D_UNAVAILABLE


def _mutated_best_option(kind):
    def f(W, L_eff, sa, sb, table, u_safe):
        ok = np.isfinite(table.s)
        r, s = table.r[ok], table.s[ok]
        ctot = ((float(L_eff) * sa.amax) * sb.amax) / r
        ss = sa.sigma * sb.sigma
        nsr = ctot / (6.0 * ss) + (ctot * ctot) / (144.0 * ss * ss)
        if kind != "no_s_term":
            nsr = nsr + (s * s) * (ctot * ctot) / (float(L_eff) * ss * ss)
        if kind == "last_on_ties":
            k = int(nsr.size - 1 - np.argmin(nsr[::-1]))
        elif kind == "argmax":
            k = int(np.argmax(nsr))
        else:
            k = int(np.argmin(nsr))
        return ct.option_at(W, L_eff, sa, sb, float(r[k]), float(s[k]), u_safe)
    return f


@pytest.mark.parametrize("kind,pin,arg", [
    ("argmax", test_best_option_zero_s_takes_largest_r, 0),
    ("no_s_term", test_best_option_matches_rational_bruteforce, 0),
    ("last_on_ties", test_best_option_tie_goes_to_first, (0.0, 1e-30)),
])
def test_best_option_mutations_fail(monkeypatch, kind, pin, arg):
    """Planted mistakes in the option choice: each makes one of the pins fail."""
    monkeypatch.setattr(ct, "best_option", _mutated_best_option(kind))
    with pytest.raises(AssertionError):
        pin(arg)


# ---------------------------------------------------------------------------
# Sec. 6: an option the calibration cannot supply is always removed

def _opts(ds_by_w):
    """options[l][W] with only the D values set (what the pruning reads)."""
    out = []
    for l in range(len(ds_by_w[1])):
        o = {}
        for W, ds in ds_by_w.items():
            o[W] = ct.PairOption(W, 0.0, 1.0, 1.0, 0.0, 0.0, 0.0, 0, 1.0, ds[l], 0.0, 0.0)
        out.append(o)
    return out


def test_accel_drops_unavailable_whatever_the_target():
    """F_kernel = 1 keeps every pair at the maximum W, except where that option is
    unavailable: such pairs drop to the next available W."""
    U = ct.D_UNAVAILABLE
    opts = _opts({4: [U, 1.0, U, 2.0], 2: [0.5, 0.3, U, 0.2], 1: [0.0] * 4})
    assert ct.prune_accel(opts, [4, 2, 1], 1.0) == [2, 4, 1, 4]
    assert ct.prune_accel(opts, [4, 2, 1], 0.0) == [1, 1, 1, 1]


def test_snr_drops_unavailable_with_infinite_budget():
    """An infinite budget (S = -inf dB) still removes unavailable options."""
    U = ct.D_UNAVAILABLE
    opts = _opts({4: [U, 1.0, 3.0], 2: [U, 0.3, 0.1], 1: [0.0] * 3})
    assert ct.prune(opts, [4, 2, 1], math.inf) == [1, 4, 4]
    assert ct.prune(opts, [4, 2, 1], 2.0) == [1, 4, 2]


def test_unavailable_rule_mutation_fails(monkeypatch):
    """Planted mistake: the throughput check applied to unavailable options too."""
    def old(options, w_desc, frac):
        nl = len(options)
        level = [0] * nl
        d = [options[l][w_desc[0]].d for l in range(nl)]
        saved = nl * ct.saved_units(w_desc[0])
        target = ct.accel_target(nl, w_desc[0], frac)
        while True:
            cand = [l for l in range(nl) if level[l] < len(w_desc) - 1]
            if not cand:
                break
            lstar = max(cand, key=lambda l: (d[l], -l))
            if not d[lstar] > 0.0:
                break
            after = saved - ct.saved_units(w_desc[level[lstar]]) + ct.saved_units(w_desc[level[lstar] + 1])
            if after < target:
                break
            saved = after
            level[lstar] += 1
            d[lstar] = options[lstar][w_desc[level[lstar]]].d
        return [w_desc[level[l]] for l in range(nl)]
    monkeypatch.setattr(ct, "prune_accel", old)
    with pytest.raises(AssertionError):
        test_accel_drops_unavailable_whatever_the_target()
