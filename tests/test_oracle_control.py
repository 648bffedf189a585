"""Pins of the oracle's plan (Sec. 5.B) and pruning (Sec. 6), and end-to-end checks.

* Pruning with W in {1, 2} has a closed characterisation that does not follow
  the greedy loop: the pairs left at W = 2 are those outside the smallest set
  of largest-D pairs whose removal brings the sum under the budget.
* Invariants for W in {1, 2, 4}: the budget is met, and undoing the last step
  breaks it; brute force over all assignments for K/L <= 4 shows the
  greedy's result is feasible whenever one is.
* Special cases: S = +inf leaves every pair at native precision and the
  result is the plain FP64 product; an all-zero block contributes nothing.
* The distortion controller meets its SNR target on i.i.d. data and its
  predicted SNR matches the measured one (Sec. 5-6, eq. 20).
* Border blocks (the cleanup of Sec. 2) give the same accuracy.
* The single-GEMM workload (256^3, L = 64, W = 2 symmetric, R = 2^20) stays in
  the exact regime: every unpacked integer equals the brute-force product.
* Fig. 7 / Sec. 7: with every pair at W = 2 in single precision, symmetric
  packing is more accurate than asymmetric packing.
"""
import dataclasses
import itertools
import math

import numpy as np
import pytest

import workloads
from oracle import control as ct
from oracle import packing as pk
from oracle import pipeline as pl
from oracle.exactsum import exact_sum
from tests.oracle_tables import tables


def _opt(W, d):
    return ct.PairOption(W, 0.0, 1.0, 1.0, 0.0, 0.0, 0.0, 0, 1.0, d, 0.0, 0.0)


def test_prune_two_levels_closed_form():
    rng = np.random.default_rng(5)
    for trial in range(300):
        n = int(rng.integers(1, 12))
        d2 = rng.exponential(1.0, n)
        if trial % 5 == 0:
            d2[rng.integers(0, n)] = d2[0]            # ties
        budget = float(rng.uniform(0, d2.sum() * 1.2))
        opts = [{2: _opt(2, float(d)), 1: _opt(1, 0.0)} for d in d2]
        got = ct.prune(opts, [2, 1], budget)
        # closed form: drop the k largest (lowest index first among equals), k minimal
        order = sorted(range(n), key=lambda l: (-d2[l], l))
        for k in range(n + 1):
            keep = set(order[k:])
            if exact_sum([d2[l] for l in keep]) <= budget:
                break
        assert got == [2 if l in keep else 1 for l in range(n)]


def test_prune_three_levels_invariants_and_bruteforce():
    rng = np.random.default_rng(9)
    for trial in range(200):
        n = int(rng.integers(1, 5))
        d2 = rng.exponential(1.0, n)
        d4 = d2 + rng.exponential(3.0, n)
        opts = [{4: _opt(4, float(d4[l])), 2: _opt(2, float(d2[l])), 1: _opt(1, 0.0)} for l in range(n)]
        budget = float(rng.uniform(0, d4.sum()))
        w = ct.prune(opts, [4, 2, 1], budget)
        tot = exact_sum([opts[l][w[l]].d for l in range(n)])
        assert tot <= budget or all(x == 1 for x in w)
        # some assignment is feasible (all W = 1 has D = 0), so the greedy result must be
        assert tot <= budget
        # the step before the last one was infeasible: raising any lowered pair back
        # by one level either exceeds the budget or was not the greedy's last move
        feasible = [a for a in itertools.product([4, 2, 1], repeat=n)
                    if exact_sum([opts[l][a[l]].d for l in range(n)]) <= budget]
        assert tuple(w) in feasible
        if all(x == 4 for x in w):
            assert exact_sum(d4.tolist()) <= budget


def test_infinite_snr_is_plain_gemm():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((128, 192))
    B = rng.standard_normal((192, 64))
    cfg = pl.Config(L=64, ctrl="snr", snr_db=float("inf"), w_allowed=(1, 2))
    res = pl.run(A, B, cfg, calib=tables(64, "sym", "f64", (2,)))
    assert all(o.W == 1 for o in res.plan.chosen.values())
    ref = A @ B
    assert np.linalg.norm(res.C - ref) / np.linalg.norm(ref) < 1e-14


def test_zero_block_contributes_nothing():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((64, 128))
    A[:, 64:] = 0.0                                   # block (0, 1) of A is all zero
    B = rng.standard_normal((128, 64))
    cfg = pl.Config(L=64, ctrl="fixed", fixed_w=2, fixed_rmax=2.0 ** 20)
    res = pl.run(A, B, cfg, keep=True)
    o = res.plan.chosen[(0, 0, 1)]
    assert o.c_a == 0.0 and o.inv == 0.0 and o.d == 0.0
    assert np.all(res.traces[(0, 0, 1)].r == 0)
    assert pl.snr_db(res.C, A @ B) > 35.0


@pytest.mark.parametrize("dist", ["gaussian", "laplace"])
@pytest.mark.parametrize("target", [20.0, 30.0, 40.0, 50.0, 60.0])
def test_snr_control_meets_target(dist, target):
    A, B = workloads.sweep(dist, n=256, k=512)
    cfg = pl.Config(L=64, ctrl="snr", snr_db=target, w_allowed=(1, 2, 4))
    res = pl.run(A, B, cfg, calib=tables(64, "sym", "f64", (2, 4)))
    got = pl.snr_db(res.C, A @ B)
    # model prediction: total signal / total expected noise over all outputs
    sig = sum(ct.signal_term(64, res.plan.stats_a[i][l], res.plan.stats_b[l][j])
              for (i, j, l) in res.plan.chosen)
    noise = sum(o.d for o in res.plan.chosen.values())
    pred = 10 * math.log10(sig / noise) if noise > 0 else float("inf")
    assert got >= target - 1.0
    # the model is conservative where the (uniform-input) representation term
    # enters; with no representation noise it is tight
    assert got >= pred - 1.0
    if all(o.s_rep == 0.0 for o in res.plan.chosen.values()):
        assert abs(got - pred) < 1.0


def test_borders_cleanup():
    rng = np.random.default_rng(8)
    A = rng.standard_normal((200, 200))
    B = rng.standard_normal((200, 72))
    cfg = pl.Config(L=64, ctrl="snr", snr_db=40.0, w_allowed=(1, 2))
    res = pl.run(A, B, cfg, calib=tables(64, "sym", "f64", (2,)))
    assert res.C.shape == (200, 72)
    assert pl.snr_db(res.C, A @ B) >= 39.0
    o = res.plan.chosen[(3, 1, 3)]                   # last l: L_eff = 200 - 192 = 8
    assert o.r_safe == 8.0 * o.q_a * o.q_b


def test_single_gemm_workload_is_exact():
    A, B = workloads.single()
    cfg = pl.Config(L=64, form="sym", prec="f64", ctrl="fixed", fixed_w=2, fixed_rmax=2.0 ** 20)
    res = pl.run(A, B, cfg, keep=True)
    assert len(res.traces) == 64
    for key, tr in res.traces.items():
        np.testing.assert_array_equal(tr.r.astype(np.int64), tr.r_exact)
        o = res.plan.chosen[key]
        assert pk.exact_regime_sym(32, o.q_a, o.q_b, 2, o.p, o.r_safe, "f64")
    # Prop. 2 prediction of the output SNR (s = 0 here)
    sig = sum(ct.signal_term(64, res.plan.stats_a[i][l], res.plan.stats_b[l][j]) for (i, j, l) in res.plan.chosen)
    noise = sum(o.d for o in res.plan.chosen.values())
    assert abs(pl.snr_db(res.C, A @ B) - 10 * math.log10(sig / noise)) < 0.5


def test_symmetric_beats_asymmetric_at_full_w2_single_precision():
    A, B = workloads.sweep("random_range", n=256)
    out = {}
    for form in ("sym", "asym"):
        cfg = pl.Config(L=64, form=form, prec="f32", ctrl="snr", snr_db=0.0, w_allowed=(1, 2))
        res = pl.run(A, B, cfg, calib=tables(64, form, "f32", (2,)))
        assert all(o.W == 2 for o in res.plan.chosen.values())
        out[form] = pl.snr_db(res.C, A @ B)
    assert out["sym"] > out["asym"]


# --- throughput-constrained pruning (F_kernel)

def test_prune_accel_two_levels_is_the_cheapest_fraction():
    """W in {1, 2}: the greedy keeps the ceil(F nL) pairs of smallest D at W = 2 (lowest l
    first among equals); brute force over all subsets of that size confirms it minimises
    the sum of D under the constraint."""
    rng = np.random.default_rng(21)
    for trial in range(200):
        n = int(rng.integers(1, 9))
        d2 = rng.exponential(1.0, n) + 0.01
        if trial % 4 == 0:
            d2[rng.integers(0, n)] = d2[0]
        frac = float(rng.choice([0.0, 0.1, 0.25, 0.5, 0.7, 1.0, rng.uniform()]))
        opts = [{2: _opt(2, float(d)), 1: _opt(1, 0.0)} for d in d2]
        got = ct.prune_accel(opts, [2, 1], frac)
        need = math.ceil(frac * n - 1e-12)
        assert sum(w == 2 for w in got) == need
        best = min(sum(d2[l] for l in keep) for keep in itertools.combinations(range(n), need))
        assert math.isclose(sum(d2[l] for l in range(n) if got[l] == 2), best, rel_tol=0, abs_tol=0)


def test_prune_accel_extremes_and_invariants():
    rng = np.random.default_rng(22)
    for trial in range(150):
        n = int(rng.integers(1, 6))
        d2 = rng.exponential(1.0, n) + 0.01
        d4 = d2 + rng.exponential(3.0, n)
        opts = [{4: _opt(4, float(d4[l])), 2: _opt(2, float(d2[l])), 1: _opt(1, 0.0)} for l in range(n)]
        assert ct.prune_accel(opts, [4, 2, 1], 1.0) == [4] * n
        assert ct.prune_accel(opts, [4, 2, 1], 0.0) == [1] * n
        frac = float(rng.uniform())
        w = ct.prune_accel(opts, [4, 2, 1], frac)
        saved = sum(ct.saved_units(x) for x in w)
        target = ct.accel_target(n, 4, frac)
        assert saved >= target
        # the next greedy move (highest current D that can still drop) would break the target
        cur = [opts[l][w[l]].d for l in range(n)]
        cand = [l for l in range(n) if w[l] != 1]
        if cand:
            l = max(cand, key=lambda x: (cur[x], -x))
            nxt = {4: 2, 2: 1}[w[l]]
            assert saved - ct.saved_units(w[l]) + ct.saved_units(nxt) < target


def test_prune_accel_keeps_zero_distortion_pairs():
    opts = [{2: _opt(2, 0.0), 1: _opt(1, 0.0)}, {2: _opt(2, 1.0), 1: _opt(1, 0.0)}]
    assert ct.prune_accel(opts, [2, 1], 0.0) == [2, 1]      # nothing to gain from the first


def test_saved_units_are_twelfths_of_the_plain_product():
    """Throughput units: a pair at packing W runs 1/W of the W = 1 MFMA work, so it
    saves 1 - 1/W of it; in twelfths this is an integer for every W dividing 12."""
    from fractions import Fraction
    for W in (1, 2, 3, 4):
        assert Fraction(ct.saved_units(W), 12) == 1 - Fraction(1, W)
    with pytest.raises(ValueError):
        ct.saved_units(5)


def test_prune_accel_three_levels_with_w3_bruteforce():
    """W in {1, 2, 3}: the result meets the constraint, the next greedy drop would
    break it, and (brute force) no assignment that meets the constraint and packs
    every pair at least as much has a smaller distortion sum."""
    rng = np.random.default_rng(23)
    for trial in range(150):
        n = int(rng.integers(1, 6))
        d2 = rng.exponential(1.0, n) + 0.01
        d3 = d2 + rng.exponential(2.0, n)
        opts = [{3: _opt(3, float(d3[l])), 2: _opt(2, float(d2[l])), 1: _opt(1, 0.0)} for l in range(n)]
        assert ct.prune_accel(opts, [3, 2, 1], 1.0) == [3] * n
        assert ct.prune_accel(opts, [3, 2, 1], 0.0) == [1] * n
        frac = float(rng.uniform())
        w = ct.prune_accel(opts, [3, 2, 1], frac)
        saved = sum(ct.saved_units(x) for x in w)
        target = ct.accel_target(n, 3, frac)
        assert saved >= target
        cur = [opts[l][w[l]].d for l in range(n)]
        cand = [l for l in range(n) if w[l] != 1]
        if cand:
            l = max(cand, key=lambda x: (cur[x], -x))
            nxt = {3: 2, 2: 1}[w[l]]
            assert saved - ct.saved_units(w[l]) + ct.saved_units(nxt) < target
        dsum = sum(cur)
        for alt in itertools.product([3, 2, 1], repeat=n):
            if sum(ct.saved_units(x) for x in alt) < target:
                continue
            if all(a >= b for a, b in zip(alt, w)) and alt != tuple(w):
                assert sum(opts[l][alt[l]].d for l in range(n)) >= dsum


def test_per_tile_targets():
    """Sec. 6: each inner kernel R_ij is pruned to its own S_kernel(i, j) (or
    F_kernel(i, j)). A uniform map equals the single target; +inf keeps a tile
    native; each tile of a mixed map equals the plan made with that tile's
    target alone."""
    rng = np.random.default_rng(31)
    A = rng.standard_normal((128, 256))
    B = rng.laplace(0.0, 1.0, (256, 192))
    calib = {W: tables(64, "sym", "f64", (2, 4))[W] for W in (2, 4)}
    base = pl.Config(L=64, form="sym", ctrl="snr", snr_db=30.0, w_allowed=(1, 2, 4))
    ref = pl.make_plan(A, B, base, calib)
    uni = pl.make_plan(A, B, dataclasses.replace(base, tile_targets=((30.0,) * 3,) * 2), calib)
    assert uni.chosen == ref.chosen and uni.budget == ref.budget
    smap = ((math.inf, 20.0, 45.0), (60.0, 30.0, 25.0))
    mixed = pl.make_plan(A, B, dataclasses.replace(base, tile_targets=smap), calib)
    assert all(mixed.chosen[(0, 0, l)].W == 1 for l in range(4))
    for i in range(2):
        for j in range(3):
            one = pl.make_plan(A, B, dataclasses.replace(base, snr_db=smap[i][j]), calib, tiles=[(i, j)])
            assert all(mixed.chosen[(i, j, l)] == one.chosen[(i, j, l)] for l in range(4))
            assert mixed.budget[(i, j)] == one.budget[(i, j)]
    fmap = ((0.0, 1.0, 0.5), (0.25, 0.75, 1.0))
    acc = dataclasses.replace(base, ctrl="accel", tile_targets=fmap)
    got = pl.make_plan(A, B, acc, calib)
    for i in range(2):
        for j in range(3):
            one = pl.make_plan(A, B, dataclasses.replace(base, ctrl="accel", accel=fmap[i][j]), calib,
                               tiles=[(i, j)])
            assert all(got.chosen[(i, j, l)] == one.chosen[(i, j, l)] for l in range(4))


# --- Prop. 3 fixed-target companders

def test_target_option_reaches_the_target():
    """Prop. 3: the eq. (22) companders give D = L s_a^2 s_b^2 10^(-S/10) (the target
    as an MSE), keep c_A c_B = 1 / c_tot (eqs. 17, 24) and, with the + root, c_A >= c_A*.
    Past eq. (25) the pair falls back to the eq. (26) companders, whose D is the
    smallest this R_max allows and lies above the target."""
    rng = np.random.default_rng(51)
    L = 64
    A = rng.standard_normal((L, L))
    B = rng.laplace(0.0, 1.0, (L, L))
    from oracle import blocks as bk
    from oracle.noise import c_tot_eq24, companders_eq26, combined_noise_eq21
    sa, sb = bk.block_stats(A, 0, 0, L), bk.block_stats(B, 0, 0, L)
    r_max = float(2 ** 16)
    ctot = c_tot_eq24(float(L), sa.amax, sb.amax, r_max)
    ca_star, cb_star = companders_eq26(sa.sigma, sb.sigma, ctot)
    d_min = combined_noise_eq21(float(L), sa.sigma, sb.sigma, ca_star, cb_star, 0.0)
    sig = float(L) * (sa.sigma * sb.sigma) ** 2
    s_max = 10.0 * math.log10(sig / d_min)
    for S in (s_max - 20.0, s_max - 6.0, s_max - 0.5):
        o = ct.target_option(2, L, sa, sb, r_max, 0.0, S, 50.0)
        assert abs(o.d / (sig * 10.0 ** (-S / 10.0)) - 1.0) < 1e-9, S
        assert abs(o.c_a * o.c_b * ctot - 1.0) < 1e-12
        assert o.c_a >= ca_star and o.c_b <= cb_star
    for S in (s_max + 0.5, s_max + 10.0, math.inf):
        o = ct.target_option(2, L, sa, sb, r_max, 0.0, S, 50.0)
        assert (o.c_a, o.c_b) == (ca_star, cb_star)
        assert o.d == d_min and o.d > sig * 10.0 ** (-S / 10.0)


def test_table_s_at_reads_the_next_grid_point():
    tab = ct.CalibTable(np.array([10.0, 20.0, 40.0, 80.0]), np.array([0.0, 0.5, np.inf, 2.0]))
    assert ct.table_s_at(tab, 5.0, 2) == 0.0
    assert ct.table_s_at(tab, 20.0, 2) == 0.5
    assert ct.table_s_at(tab, 21.0, 2) == math.inf
    assert ct.table_s_at(tab, 41.0, 2) == 2.0
    assert ct.table_s_at(tab, 81.0, 2) == math.inf


def test_target_control_meets_the_subblock_snr():
    """End to end: every pair set by Prop. 3 to S dB; the measured SNR of C against the
    FP64 product is S within the model's accuracy (exact-regime integers, W = 2)."""
    rng = np.random.default_rng(52)
    A = rng.standard_normal((256, 256))
    B = rng.standard_normal((256, 256))
    calib = {2: tables(64, "sym", "f64", (2,))[2]}
    ref = A @ B
    got = {}
    for S in (25.0, 40.0, 70.0):
        cfg = pl.Config(L=64, form="sym", ctrl="target", snr_db=S, w_allowed=(1, 2), fixed_w=2,
                        fixed_rmax=float(2 ** 22))
        got[S] = pl.snr_db(pl.run(A, B, cfg, calib=calib).C, ref)
    assert abs(got[25.0] - 25.0) < 1.0 and abs(got[40.0] - 40.0) < 1.0, got
    assert 40.0 < got[70.0] < 50.0, got          # beyond reach: the best R_max = 2^22 allows


def test_grouped_l_sum():
    """The l-sum of eq. (2) in groups of consecutive subblocks: one group is the plain
    ascending sum bit for bit; any grouping stays within FP64 rounding of it and every
    group size is ceil(nL / k_groups)."""
    rng = np.random.default_rng(61)
    A = rng.standard_normal((96, 64 * 9))
    B = rng.laplace(0.0, 1.0, (64 * 9, 80))
    calib = {W: tables(64, "sym", "f64", (2, 4))[W] for W in (2, 4)}
    cfg = pl.Config(L=64, form="sym", ctrl="snr", snr_db=30.0, w_allowed=(1, 2, 4))
    plan = pl.make_plan(A, B, cfg, calib)
    one = pl.run(A, B, cfg, calib, plan=plan).C
    assert np.array_equal(pl.run(A, B, dataclasses.replace(cfg, k_groups=1), calib, plan=plan).C, one)
    for G, size in ((2, 5), (3, 3), (4, 3), (9, 1), (20, 1)):
        assert pl.group_size(9, G) == size
        got = pl.run(A, B, dataclasses.replace(cfg, k_groups=G), calib, plan=plan).C
        assert np.max(np.abs(got - one)) <= 1e-12 * np.max(np.abs(one))
    with pytest.raises(ValueError):
        pl.group_size(9, 0)


def test_accel_units_from_measured_accelerations():
    """Sec. 5.B keeps the measured acceleration F_W of each packing: a pair at W
    saves 1 - 1/F_W of its W = 1 time, quantised to integer units."""
    u = ct.accel_units({2: 2.0, 3: 4.0 / 3.0, 4: 1.0, 5: 0.8}, scale=4096)
    assert u == {2: 2048, 3: 1024, 4: 0, 5: 0}
    assert ct.saved_units(1, u) == 0 and ct.saved_units(3, u) == 1024


@pytest.mark.parametrize("u2,u4", [(1365, 2000), (1365, 1000), (2048, 3072), (500, 500)])
def test_prune_accel_with_measured_units(u2, u4):
    """With measured units (W = 4 may save more or less than W = 2): the result
    meets the constraint, and the greedy's next move (the highest current D that
    can still drop) would either break it or gain time; W in {1, 2} keeps the
    fraction of packed pairs whatever the unit."""
    rng = np.random.default_rng(u2 + u4)
    units = {2: u2, 4: u4}
    for trial in range(150):
        n = int(rng.integers(1, 7))
        d2 = rng.exponential(1.0, n) + 0.01
        d4 = d2 + rng.exponential(3.0, n)
        opts = [{4: _opt(4, float(d4[l])), 2: _opt(2, float(d2[l])), 1: _opt(1, 0.0)} for l in range(n)]
        frac = float(rng.uniform())
        w = ct.prune_accel(opts, [4, 2, 1], frac, units)
        saved = sum(ct.saved_units(x, units) for x in w)
        target = ct.accel_target(n, 4, frac, units)
        assert saved >= target
        cur = [opts[l][w[l]].d for l in range(n)]
        cand = [l for l in range(n) if w[l] != 1]
        if cand:
            l = max(cand, key=lambda x: (cur[x], -x))
            nxt = {4: 2, 2: 1}[w[l]]
            assert saved - ct.saved_units(w[l], units) + ct.saved_units(nxt, units) < target
        two = [{2: _opt(2, float(d2[l])), 1: _opt(1, 0.0)} for l in range(n)]
        assert ct.prune_accel(two, [2, 1], frac, units) == ct.prune_accel(two, [2, 1], frac)
