"""GPU parity of the plan alone (statistics, per-pair options, Sec. 6 pruning)
on inputs chosen to stress the pruning: equal noise values across subblocks,
more than 64 subblocks along K, calibration tables under which D does not
decrease with W (the step-by-step greedy) and tables with no usable W = 4
point. Records and budgets must equal the oracle's bit for bit."""
import math
import zlib

import numpy as np
import pytest

from oracle import control as ct
from oracle import pipeline as pl
from tests.gpu_common import compare_plan, log, oracle_cfg, to_dev
from tests.oracle_tables import tables

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def td():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1110_5765_amd import tdgemm
    return tdgemm


def _wmax(L):
    return 3 if L == 96 else 4


def _calib(kind, L, form):
    tabs = tables(L, form, "f64", (2, 3, 4) if L == 96 else (2, 4))
    r = tabs[2].r
    if kind == "scaled_w4":          # W = 4 cheaper than W = 2: D need not fall with W
        tabs = {2: tabs[2], 4: ct.CalibTable(r.copy(), tabs[2].s * 0.25)}
    elif kind == "no_w4":            # no usable W = 4 point: D_4 is the "unavailable" value
        tabs = {2: tabs[2], 4: ct.CalibTable(r.copy(), np.full(r.size, np.inf))}
    return tabs


CASES = [
    # name, M, K, N, L, form, snr, w_allowed, inputs, calib
    ("ties_equal_blocks", 128, 384, 128, 64, "sym", 83.0, (1, 2, 4), "tiled", "std"),
    ("many_l_T2", 128, 64 * 70, 128, 64, "sym", 30.0, (1, 2, 4), "gauss", "std"),
    ("many_l_T5_ragged", 64, 64 * 300 + 17, 70, 64, "asym", 25.0, (1, 2, 4), "laplace", "std"),
    ("L128_many_l", 128, 128 * 70, 128, 128, "sym", 35.0, (1, 2, 4), "gauss", "std"),
    ("nonmono_fallback", 192, 640, 128, 64, "sym", 86.0, (1, 2, 4), "gauss", "scaled_w4"),
    ("unavailable_w4", 128, 512, 192, 64, "sym", 80.0, (1, 2, 4), "laplace", "no_w4"),
    ("deep_prune_w2_only", 256, 1024, 64, 64, "sym", 80.0, (1, 2), "laplace", "std"),
    ("L96_many_l", 96, 96 * 70, 96, 96, "sym", 30.0, (1, 2, 3), "gauss", "std"),
    ("L96_asym_ragged", 64, 96 * 50 + 17, 70, 96, "asym", 25.0, (1, 2, 3), "laplace", "std"),
    ("L96_w1234_many_l", 96, 96 * 70, 96, 96, "sym", 22.0, (1, 2, 3, 4), "gauss", "std"),
    # four subblocks per lane: one workgroup per inner kernel, four wavefronts ranking
    ("T4_w124_ragged", 64, 64 * 200 + 5, 128, 64, "sym", 30.0, (1, 2, 4), "gauss", "std"),
    ("T3_nonmono_fallback", 64, 64 * 150, 128, 64, "sym", 86.0, (1, 2, 4), "gauss", "scaled_w4"),
]


def _inputs(kind, M, K, N, seed):
    r = np.random.default_rng(seed)
    if kind == "tiled":              # the same 64 x 64 block repeated along K
        a = r.standard_normal((M, 64))
        b = r.standard_normal((64, N))
        return np.tile(a, (1, K // 64)), np.tile(b, (K // 64, 1))
    if kind == "gauss":
        return r.standard_normal((M, K)), r.standard_normal((K, N))
    A = r.laplace(0.0, 1.0, (M, K)) * (1.0 + 4.0 * r.random((1, K)))   # uneven column scales
    return A, r.laplace(0.0, 1.0, (K, N))


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_plan_parity(td, case):
    name, M, K, N, L, form, snr, wal, kind, ckind = case
    log(f"[plan] {name}: M={M} K={K} N={N} L={L} {form} snr={snr} calib={ckind}")
    A, B = _inputs(kind, M, K, N, zlib.crc32(name.encode()))
    tabs = _calib(ckind, L, form)
    cfg = oracle_cfg(L, form, "f64", "snr", snr, wal, 2, 1.0, 127.0)
    ref = pl.make_plan(A, B, cfg, calib=tabs)
    calib = td.DeviceCalib(tabs[2].r, {W: t.s for W, t in tabs.items()})
    Ad, Bd = to_dev(A), to_dev(B)
    desc = td.make_desc(Ad, Bd, L=L, form=form, prec="f64", ctrl="snr", snr_db=snr, w_allowed=wal)
    plan = td.tdgemm_plan(desc, Ad, Bd, calib)
    sa, sb, pairs, budget = td.tdgemm_plan_export(plan)
    nI, nL, nJ, _ = plan.dims

    class _Res:
        pass
    res = _Res()
    res.plan = ref
    compare_plan(pairs, budget, sa, sb, res, [(i, j) for i in range(nI) for j in range(nJ)])
    ws = np.bincount(pairs["w"].ravel(), minlength=5)
    log(f"[plan] {name}: W histogram {ws.tolist()}")
    if name == "ties_equal_blocks":   # equal D everywhere: pruned pairs are the lowest l
        w = pairs["w"]
        for i in range(nI):
            for j in range(nJ):
                row = w[i, j]
                assert all(row[l] <= row[l + 1] for l in range(nL - 1)), row


ACCEL_CASES = [
    # name, M, K, N, L, form, frac, w_allowed, inputs, calib
    ("accel_w2_f0", 128, 384, 128, 64, "sym", 0.0, (1, 2), "laplace", "std"),
    ("accel_w2_f03", 192, 640, 128, 64, "sym", 0.3, (1, 2), "gauss", "std"),
    ("accel_w2_f05_asym", 128, 512, 192, 64, "asym", 0.5, (1, 2), "laplace", "std"),
    ("accel_w2_f1", 128, 384, 128, 64, "sym", 1.0, (1, 2), "gauss", "std"),
    ("accel_w24_f06", 256, 1024, 64, 64, "sym", 0.6, (1, 2, 4), "laplace", "std"),
    ("accel_L128_many_l", 128, 128 * 70, 128, 128, "sym", 0.45, (1, 2, 4), "gauss", "std"),
    ("accel_ties", 128, 384, 128, 64, "sym", 0.5, (1, 2), "tiled", "std"),
    ("accel_L96_w23", 192, 96 * 20, 96, 96, "sym", 0.55, (1, 2, 3), "laplace", "std"),
    ("accel_L96_asym", 96, 96 * 12, 192, 96, "asym", 0.3, (1, 2, 3), "gauss", "std"),
    ("accel_L96_w1234", 192, 96 * 20, 96, 96, "sym", 0.6, (1, 2, 3, 4), "laplace", "std"),
    ("accel_nonmono_fallback", 192, 640, 128, 64, "sym", 0.5, (1, 2, 4), "gauss", "scaled_w4"),
    ("accel_T4_w124", 64, 64 * 230, 128, 64, "sym", 0.6, (1, 2, 4), "laplace", "std"),
]


@pytest.mark.parametrize("case", ACCEL_CASES, ids=[c[0] for c in ACCEL_CASES])
def test_accel_plan_parity(td, case):
    """Throughput-constrained pruning (F_kernel): records bit-exact to the oracle."""
    name, M, K, N, L, form, frac, wal, kind, ck = case
    log(f"[plan] {name}: M={M} K={K} N={N} L={L} {form} F={frac} W={wal} calib {ck}")
    A, B = _inputs(kind, M, K, N, zlib.crc32(name.encode()))
    tabs = _calib(ck, L, form)
    cfg = pl.Config(L=L, form=form, prec="f64", ctrl="accel", accel=frac, w_allowed=tuple(wal))
    ref = pl.make_plan(A, B, cfg, calib=tabs)
    calib = td.DeviceCalib(tabs[2].r, {W: t.s for W, t in tabs.items()})
    Ad, Bd = to_dev(A), to_dev(B)
    desc = td.make_desc(Ad, Bd, L=L, form=form, prec="f64", ctrl="accel", accel=frac, w_allowed=wal)
    plan = td.tdgemm_plan(desc, Ad, Bd, calib)
    sa, sb, pairs, budget = td.tdgemm_plan_export(plan)
    nI, nL, nJ, _ = plan.dims

    class _Res:
        pass
    res = _Res()
    res.plan = ref
    compare_plan(pairs, budget, sa, sb, res, [(i, j) for i in range(nI) for j in range(nJ)])
    ws = np.bincount(pairs["w"].ravel(), minlength=5)
    log(f"[plan] {name}: W histogram {ws.tolist()}")
    if name == "accel_w2_f05_asym":          # the product too
        C = torch.empty((M, N), dtype=torch.float64, device="cuda")
        td.tdgemm_gemm(plan, Ad, Bd, C, fused=1)
        Cref = pl.run(A, B, cfg, calib=tabs, plan=ref).C
        got = C.cpu().numpy()
        assert float(np.linalg.norm(got - Cref) / np.linalg.norm(Cref)) <= 1e-12


@pytest.mark.parametrize("ctrl,L,form", [("snr", 64, "sym"), ("snr", 96, "asym"), ("accel", 128, "sym"),
                                         ("target", 64, "asym")])
def test_tile_target_plan_parity(td, ctrl, L, form):
    """Per-inner-kernel targets S_kernel(i, j) / F_kernel(i, j) (Sec. 6), and per-tile
    subblock targets of the Prop. 3 control: records and
    budgets bit-exact to the oracle, and the product of the packed path."""
    M, K, N = 5 * L - 17, 4 * L, 4 * L + 9
    nI, nJ = -(-M // L), -(-N // L)
    rng = np.random.default_rng(41 + L)
    if ctrl == "snr":
        tmap = rng.choice([math.inf, 70.0, 45.0, 30.0, 22.0, 15.0], size=(nI, nJ))
    elif ctrl == "target":
        tmap = rng.choice([math.inf, 50.0, 35.0, 25.0, 15.0], size=(nI, nJ))
    else:
        tmap = rng.choice([0.0, 0.2, 0.5, 0.8, 1.0], size=(nI, nJ))
    log(f"[plan] tile targets {ctrl} L={L} {form}: {nI} x {nJ}")
    A, B = _inputs("laplace", M, K, N, 77 + L)
    tabs = _calib("std", L, form)
    wal = (1, 2, _wmax(L))
    cfg = pl.Config(L=L, form=form, prec="f64", ctrl=ctrl, snr_db=40.0, w_allowed=wal, fixed_w=2,
                    fixed_rmax=float(2 ** 20),
                    tile_targets=tuple(tuple(float(v) for v in row) for row in tmap))
    ref = pl.make_plan(A, B, cfg, calib=tabs)
    calib = td.DeviceCalib(tabs[2].r, {W: t.s for W, t in tabs.items()})
    Ad, Bd = to_dev(A), to_dev(B)
    desc = td.make_desc(Ad, Bd, L=L, form=form, prec="f64", ctrl=ctrl, snr_db=40.0, w_allowed=wal,
                        fixed_w=2, fixed_rmax=float(2 ** 20), tile_target=tmap)
    plan = td.tdgemm_plan(desc, Ad, Bd, calib)
    sa, sb, pairs, budget = td.tdgemm_plan_export(plan)

    class _Res:
        pass
    res = _Res()
    res.plan = ref
    compare_plan(pairs, budget, sa, sb, res, [(i, j) for i in range(nI) for j in range(nJ)])
    if ctrl == "snr":
        assert np.all(pairs["w"][tmap == math.inf] == 1)
    C = torch.empty((M, N), dtype=torch.float64, device="cuda")
    td.tdgemm_gemm(plan, Ad, Bd, C, fused=1)
    Cref = pl.run(A, B, cfg, calib=tabs, plan=ref).C
    got = C.cpu().numpy()
    assert float(np.linalg.norm(got - Cref) / np.linalg.norm(Cref)) <= 1e-12
    log(f"[plan] tile targets {ctrl}: W histogram {np.bincount(pairs['w'].ravel(), minlength=5).tolist()}")


QUERY_CASES = [
    # name, control, L, form, S (dB), per-tile targets
    ("snr_L64_sym", "snr", 64, "sym", 30.0, False),
    ("fixed_L128_asym", "fixed", 128, "asym", 0.0, False),
    ("target_L96_sym_map", "target", 96, "sym", 40.0, True),
    ("target_L64_asym_high", "target", 64, "asym", 75.0, False),
]


@pytest.mark.parametrize("case", QUERY_CASES, ids=[c[0] for c in QUERY_CASES])
def test_plan_query_vs_oracle(td, case):
    """tdgemm_plan_query against the oracle's own plan: the W histogram exactly,
    the predicted output SNR (signal L_eff sigma_a^2 sigma_b^2 over D, summed over
    all pairs) within 1e-9 dB, and the TARGET pairs short of their target."""
    name, ctrl, L, form, snr, per_tile = case
    M, K, N = 4 * L - 5, 5 * L + 3, 3 * L + 7
    nI, nL, nJ = -(-M // L), -(-K // L), -(-N // L)
    log(f"[plan] query {name}: M={M} K={K} N={N}")
    A, B = _inputs("laplace", M, K, N, 91 + L)
    tabs = _calib("std", L, form)
    wal = (1, 2, _wmax(L))
    fw = 3 if L == 96 else 2
    rmax = float(2 ** 14) if L == 96 else float(2 ** 20)
    tmap = None
    if per_tile:
        tmap = np.random.default_rng(5).choice([math.inf, 60.0, 40.0, 20.0], size=(nI, nJ))
    cfg = pl.Config(L=L, form=form, prec="f64", ctrl=ctrl, snr_db=snr, w_allowed=wal, fixed_w=fw,
                    fixed_rmax=rmax,
                    tile_targets=None if tmap is None else tuple(tuple(float(v) for v in r) for r in tmap))
    ref = pl.make_plan(A, B, cfg, calib=tabs)
    calib = td.DeviceCalib(tabs[2].r, {W: t.s for W, t in tabs.items()})
    Ad, Bd = to_dev(A), to_dev(B)
    desc = td.make_desc(Ad, Bd, L=L, form=form, prec="f64", ctrl=ctrl, snr_db=snr, w_allowed=wal,
                        fixed_w=fw, fixed_rmax=rmax, tile_target=tmap)
    plan = td.tdgemm_plan(desc, Ad, Bd, calib if ctrl in ("snr", "target") else None)
    got_snr, got_hist, got_short = td.tdgemm_plan_query(plan)

    sig, noise, hist, short = [], [], np.zeros(5, dtype=np.int64), 0
    for i in range(nI):
        for j in range(nJ):
            want = 10.0 ** ((tmap[i, j] if tmap is not None else snr) / 10.0)
            for l in range(nL):
                o = ref.chosen[(i, j, l)]
                sa, sb = ref.stats_a[i][l], ref.stats_b[l][j]
                va = sa.sumsq / sa.n if sa.n else 0.0
                vb = sb.sumsq / sb.n if sb.n else 0.0
                s = min(L, K - l * L) * va * vb
                sig.append(s)
                noise.append(o.d)
                hist[o.W] += 1
                if ctrl == "target" and o.W > 1 and o.d > 0.0 and s < want * o.d * (1.0 - 1e-9):
                    short += 1
    assert got_hist.tolist() == hist.tolist()
    assert got_short == short
    n_sum = math.fsum(noise)
    want_snr = math.inf if n_sum == 0.0 else 10.0 * math.log10(math.fsum(sig) / n_sum)
    assert (got_snr == want_snr) if math.isinf(want_snr) else abs(got_snr - want_snr) <= 1e-9
    log(f"[plan] query {name}: predicted SNR {got_snr:.3f} dB, W {got_hist.tolist()}, short {got_short}")


@pytest.mark.parametrize("dt", [np.float64, np.float32], ids=["f64", "f32"])
def test_sums_at_rounding_boundaries(td, dt):
    """Exactly rounded sums by construction (statistics and the Sec. 6 budget).
    Block (0, 0) of A holds 1, 2^-27, 2^-27, 2^-100: its exact sum of squares
    1 + 2^-53 + 2^-200 lies just above the midpoint between 1 and 1 + 2^-52 and
    rounds up; block (0, 1) holds 1, 2^-27, 2^-27 (an exact tie, to even: 1).
    The single inner kernel's signal terms L s_a^2 s_b^2 are 1, 2^-54, 2^-54,
    2^-200 (one nonzero element per block of A row 1 and B column 1), whose sum
    rounds up too. A compensated sum rounded once gives 1 in both cases. Block
    (0, 1) is settled by the exact compensated pair (every addition into the
    correction is exact), block (0, 0) only by the long accumulator. Every value
    is a float32 too: with float32 inputs the first pass sums the squares as
    exact compensated pairs already."""
    L, M, K, N = 64, 128, 4 * 64, 128
    rng = np.random.default_rng(2024)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    A[:64, :64] = 0.0
    A[0, :4] = [1.0, 2.0 ** -27, 2.0 ** -27, 2.0 ** -100]
    A[:64, 64:128] = 0.0
    A[5, 64:67] = [1.0, 2.0 ** -27, 2.0 ** -27]
    # inner kernel (1, 1): A row block 1 and B column block 1 with one nonzero per block
    ab = [(2.0 ** 9, 1.0), (2.0 ** -9, 2.0 ** -9), (2.0 ** -9, 2.0 ** -9), (2.0 ** -45, 2.0 ** -46)]
    A[64:, :] = 0.0
    B[:, 64:] = 0.0
    for l, (a, b) in enumerate(ab):
        A[64 + 3, l * 64 + 7] = a
        B[l * 64 + 11, 64 + 2] = b
    A, B = A.astype(dt), B.astype(dt)
    tabs = _calib("std", L, "sym")
    cfg = oracle_cfg(L, "sym", "f64", "snr", 30.0, (1, 2), 2, 1.0, 127.0)
    ref = pl.make_plan(A, B, cfg, calib=tabs)
    assert ref.stats_a[0][0].sumsq == 1.0 + 2.0 ** -52
    assert ref.stats_a[0][1].sumsq == 1.0
    terms = [ct.signal_term(L, ref.stats_a[1][l], ref.stats_b[l][1]) for l in range(4)]
    assert terms == [1.0, 2.0 ** -54, 2.0 ** -54, 2.0 ** -200]
    assert ref.budget[(1, 1)] == 10.0 ** (-3.0) * (1.0 + 2.0 ** -52)
    calib = td.DeviceCalib(tabs[2].r, {2: tabs[2].s})
    Ad, Bd = to_dev(A), to_dev(B)
    desc = td.make_desc(Ad, Bd, L=L, form="sym", prec="f64", ctrl="snr", snr_db=30.0, w_allowed=(1, 2))
    plan = td.tdgemm_plan(desc, Ad, Bd, calib)
    sa, sb, pairs, budget = td.tdgemm_plan_export(plan)
    assert sa[0, 0]["sumsq"] == 1.0 + 2.0 ** -52 and sa[0, 1]["sumsq"] == 1.0
    assert budget[1, 1] == ref.budget[(1, 1)]

    class _Res:
        pass
    res = _Res()
    res.plan = ref
    compare_plan(pairs, budget, sa, sb, res, [(i, j) for i in range(2) for j in range(2)])
    log("[plan] rounding-boundary sums: statistics and budget equal the exactly rounded values")


@pytest.mark.parametrize("ctrl,target", [("accel", 1.0), ("snr", -math.inf)])
def test_unavailable_option_always_dropped(td, ctrl, target):
    """A calibration table with no usable W = 4 point: however loose the target
    (F_kernel = 1, or S = -inf dB, an infinite budget), no pair may keep the
    unavailable W = 4 option, whose product would add nothing to C. Records equal
    the oracle's; C equals the oracle's bit for bit and stays close to A B."""
    L, M, K, N = 64, 192, 6 * 64, 128
    log(f"[plan] unavailable W = 4 under {ctrl} {target}")
    A, B = _inputs("laplace", M, K, N, 515)
    tabs = _calib("no_w4", L, "sym")
    cfg = pl.Config(L=L, form="sym", prec="f64", ctrl=ctrl, snr_db=target, accel=target,
                    w_allowed=(1, 2, 4))
    ref = pl.make_plan(A, B, cfg, calib=tabs)
    calib = td.DeviceCalib(tabs[2].r, {2: tabs[2].s, 4: tabs[4].s})
    Ad, Bd = to_dev(A), to_dev(B)
    desc = td.make_desc(Ad, Bd, L=L, form="sym", prec="f64", ctrl=ctrl, snr_db=target, accel=target,
                        w_allowed=(1, 2, 4))
    plan = td.tdgemm_plan(desc, Ad, Bd, calib)
    sa, sb, pairs, budget = td.tdgemm_plan_export(plan)

    class _Res:
        pass
    res = _Res()
    res.plan = ref
    nI, nL, nJ, _ = plan.dims
    compare_plan(pairs, budget, sa, sb, res, [(i, j) for i in range(nI) for j in range(nJ)])
    assert not np.any(pairs["w"] == 4)
    assert np.all(pairs["d"] < ct.D_UNAVAILABLE)
    C = torch.empty((M, N), dtype=torch.float64, device="cuda")
    td.tdgemm_gemm(plan, Ad, Bd, C, fused=1)
    got = C.cpu().numpy()
    np.testing.assert_array_equal(got, pl.run(A, B, cfg, calib=tabs, plan=ref).C)
    snr = pl.snr_db(got, A @ B)
    log(f"[plan] unavailable W = 4 under {ctrl}: W {np.bincount(pairs['w'].ravel(), minlength=5).tolist()}, "
        f"SNR {snr:.1f} dB")
    assert snr > 25.0


@pytest.mark.parametrize("units,frac", [({2: 1365, 4: 1800}, 0.6), ({2: 1365, 4: 900}, 0.8),
                                        ({2: 2048, 4: 3072}, 0.35)])
def test_accel_measured_units_parity(td, units, frac):
    """Throughput control with measured saved-time units per packing (Sec. 5.B F_W):
    records bit-exact to the oracle fed the same units, and the product too."""
    L, M, K, N = 64, 192, 10 * 64, 128
    log(f"[plan] ACCEL with measured units {units}, F = {frac}")
    A, B = _inputs("laplace", M, K, N, 600 + units[4])
    tabs = _calib("std", L, "sym")
    cfg = pl.Config(L=L, form="sym", prec="f64", ctrl="accel", accel=frac, w_allowed=(1, 2, 4),
                    accel_units=tuple(sorted(units.items())))
    ref = pl.make_plan(A, B, cfg, calib=tabs)
    calib = td.DeviceCalib(tabs[2].r, {2: tabs[2].s, 4: tabs[4].s})
    Ad, Bd = to_dev(A), to_dev(B)
    desc = td.make_desc(Ad, Bd, L=L, form="sym", prec="f64", ctrl="accel", accel=frac, w_allowed=(1, 2, 4),
                        accel_units=units)
    plan = td.tdgemm_plan(desc, Ad, Bd, calib)
    sa, sb, pairs, budget = td.tdgemm_plan_export(plan)

    class _Res:
        pass
    res = _Res()
    res.plan = ref
    nI, nL, nJ, _ = plan.dims
    compare_plan(pairs, budget, sa, sb, res, [(i, j) for i in range(nI) for j in range(nJ)])
    nominal = pl.make_plan(A, B, pl.Config(L=L, form="sym", prec="f64", ctrl="accel", accel=frac,
                                           w_allowed=(1, 2, 4)), calib=tabs)
    differ = sum(ref.chosen[k].W != nominal.chosen[k].W for k in ref.chosen)
    C = torch.empty((M, N), dtype=torch.float64, device="cuda")
    td.tdgemm_gemm(plan, Ad, Bd, C, fused=1)
    np.testing.assert_array_equal(C.cpu().numpy(), pl.run(A, B, cfg, calib=tabs, plan=ref).C)
    log(f"[plan] measured units: W {np.bincount(pairs['w'].ravel(), minlength=5).tolist()}, "
        f"{differ} pairs differ from the nominal-unit plan")


def test_measured_accelerations(td):
    """F_W measured on the GPU path (Sec. 5.B): packing saves time at W = 2 and 4
    (L = 128, symmetric, FP64), and a plan with the derived units matches the oracle."""
    from paper_1110_5765_amd import calib as cb
    f = cb.measure_accel(128, "sym", "f64", (2, 4), n=2048, reps=5)
    units = cb.accel_units(f)
    log(f"[plan] measured F_W at L = 128 sym f64, 2048^3: {f}, units {units}")
    assert all(1.0 < f[W] < 2.0 * W for W in (2, 4))
    assert all(units[W] > 0 for W in (2, 4))
