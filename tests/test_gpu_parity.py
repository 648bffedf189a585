"""GPU parity: the HIP path, called through the C-ABI, against the CPU oracle.

Bar (integer and byte work bit-exact; floating point within the stated bound):
* block statistics, pair records (W, p, companders, D, R, s) and budgets: bit-exact;
* companded integers, packed words, packed products and unpacked integers:
  bit-exact (the packed products are FMA chains in ascending packed index on
  both sides: the matrix cores accumulate exactly that way);
* C: equal to the oracle's element by element (bit for bit: both sides sum
  r * inv over l ascending in the same operations), the fused kernel equal to
  the staged path bit for bit, and the relative Frobenius error (<= 1e-12 FP64,
  1e-5 FP32 packing) logged as the summary. A grouped l-sum (k_split) equals the
  oracle with the same grouping bit for bit, and the oracle's plain ascending
  sum within 1e-12 / 1e-5 of |A||B| element by element.
Shapes span several tiles and ragged tails on every axis; both packing forms,
all three block sizes (L = 96 with W in {1, 2, 3, 4}), all control modes, transposed operands and the empty
and single-row cases are covered.
"""
import math
import zlib

import numpy as np
import pytest

import workloads
from oracle import pipeline as pl
from tests.gpu_common import assert_elementwise, compare_plan, device_calib, log, oracle_cfg, rel_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def td():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1110_5765_amd import tdgemm
    return tdgemm


TOL = {"f64": 1e-12, "f32": 1e-5}

CASES = [
    # name, M, K, N, L, form, in, prec, ctrl, snr, w_allowed, fixed_w, ta, tb
    ("single_sym_fixed", 256, 256, 256, 64, "sym", "f64", "f64", "fixed", 0.0, (1, 2), 2, 0, 0),
    ("ragged_sym_snr40", 200, 330, 150, 64, "sym", "f64", "f64", "snr", 40.0, (1, 2, 4), 2, 0, 0),
    ("ragged_asym_snr40", 200, 330, 150, 64, "asym", "f64", "f64", "snr", 40.0, (1, 2, 4), 2, 0, 0),
    ("sym_snr20_w4", 192, 256, 128, 64, "sym", "f64", "f64", "snr", 20.0, (1, 2, 4), 2, 0, 0),
    ("asym_snr20_w4", 192, 256, 128, 64, "asym", "f64", "f64", "snr", 20.0, (1, 2, 4), 2, 0, 0),
    ("sym_snr60", 128, 384, 128, 64, "sym", "f64", "f64", "snr", 60.0, (1, 2), 2, 0, 0),
    ("sym_inf_native", 130, 200, 70, 64, "sym", "f64", "f64", "snr", math.inf, (1, 2), 2, 0, 0),
    ("L128_sym", 300, 400, 260, 128, "sym", "f64", "f64", "snr", 40.0, (1, 2, 4), 2, 0, 0),
    ("L128_asym", 300, 400, 260, 128, "asym", "f64", "f64", "snr", 40.0, (1, 2, 4), 2, 0, 0),
    ("L128_asym_w4", 256, 256, 256, 128, "asym", "f64", "f64", "fixed", 0.0, (1, 4), 4, 0, 0),
    ("trans_a", 150, 200, 90, 64, "sym", "f64", "f64", "snr", 40.0, (1, 2), 2, 1, 0),
    ("trans_b", 150, 200, 90, 64, "asym", "f64", "f64", "snr", 40.0, (1, 2), 2, 0, 1),
    ("trans_ab_L128", 150, 200, 90, 128, "sym", "f64", "f64", "snr", 40.0, (1, 2), 2, 1, 1),
    ("f32_in_f64_pack", 200, 300, 100, 64, "sym", "f32", "f64", "snr", 40.0, (1, 2), 2, 0, 0),
    ("f32_pack_sym", 200, 300, 100, 64, "sym", "f32", "f32", "snr", 15.0, (1, 2), 2, 0, 0),
    ("f32_pack_asym_L128", 200, 300, 160, 128, "asym", "f32", "f32", "snr", 10.0, (1, 2), 2, 0, 0),
    # the instantiations the scatter (FP32 in, FP64 packing, A transposed) and the
    # perceptron (FP32 packing, either operand transposed) workloads run at L = 128
    ("L128_f32_in_f64_ta", 300, 260, 280, 128, "sym", "f32", "f64", "snr", 40.0, (1, 2, 4), 2, 1, 0),
    ("L128_f32_in_f64_asym", 200, 300, 150, 128, "asym", "f32", "f64", "snr", 30.0, (1, 2, 4), 2, 0, 0),
    ("L128_f32_pack_sym_ta", 260, 300, 140, 128, "sym", "f32", "f32", "snr", 15.0, (1, 2), 2, 1, 0),
    ("L128_f32_pack_sym_tb", 200, 300, 160, 128, "sym", "f32", "f32", "snr", 15.0, (1, 2), 2, 0, 1),
    ("separable_q127", 256, 256, 192, 128, "sym", "f64", "f64", "separable", 0.0, (1, 2), 2, 0, 0),
    ("single_row", 1, 100, 70, 64, "sym", "f64", "f64", "snr", 40.0, (1, 2), 2, 0, 0),
    ("k_below_L", 70, 20, 90, 64, "asym", "f64", "f64", "snr", 30.0, (1, 2, 4), 2, 0, 0),
    # Prop. 3 control: a target subblock SNR per pair (the second is out of reach)
    ("target_sym_s30", 200, 330, 150, 64, "sym", "f64", "f64", "target", 30.0, (1, 2), 2, 0, 0),
    ("target_asym_s60_capped", 200, 330, 150, 64, "asym", "f64", "f64", "target", 60.0, (1, 2), 2, 0, 0),
    ("target_L96_w3", 192, 288, 200, 96, "sym", "f64", "f64", "target", 12.0, (1, 3), 3, 0, 0),
    # L = 96: packings {1, 2, 3}
    ("L96_sym_snr30_w3", 300, 400, 260, 96, "sym", "f64", "f64", "snr", 30.0, (1, 2, 3), 2, 0, 0),
    ("L96_asym_snr30_w3", 300, 400, 260, 96, "asym", "f64", "f64", "snr", 30.0, (1, 2, 3), 2, 0, 0),
    ("L96_sym_fixed_w3", 200, 288, 200, 96, "sym", "f64", "f64", "fixed", 0.0, (1, 3), 3, 0, 0),
    ("L96_asym_fixed_w3", 200, 288, 200, 96, "asym", "f64", "f64", "fixed", 0.0, (1, 3), 3, 0, 0),
    ("L96_asym_snr50", 192, 300, 96, 96, "asym", "f64", "f64", "snr", 50.0, (1, 2, 3), 2, 0, 0),
    ("L96_trans_ab", 150, 200, 90, 96, "asym", "f64", "f64", "snr", 30.0, (1, 2, 3), 2, 1, 1),
    ("L96_trans_a_sym", 150, 200, 90, 96, "sym", "f64", "f64", "snr", 30.0, (1, 2, 3), 2, 1, 0),
    ("L96_f32_in", 200, 300, 100, 96, "sym", "f32", "f64", "snr", 40.0, (1, 2, 3), 2, 0, 0),
    ("L96_f32_pack_sym", 200, 300, 100, 96, "sym", "f32", "f32", "snr", 15.0, (1, 2), 2, 0, 0),
    ("L96_f32_pack_asym", 200, 300, 100, 96, "asym", "f32", "f32", "snr", 10.0, (1, 2), 2, 0, 0),
    ("L96_separable_w3", 192, 192, 192, 96, "sym", "f64", "f64", "separable", 0.0, (1, 3), 3, 0, 0),
    # L = 96 with the whole double-precision set {1, 2, 3, 4} (48-column chunks)
    ("L96_sym_fixed_w4", 200, 288, 200, 96, "sym", "f64", "f64", "fixed", 0.0, (1, 4), 4, 0, 0),
    ("L96_asym_fixed_w4", 200, 288, 200, 96, "asym", "f64", "f64", "fixed", 0.0, (1, 4), 4, 0, 0),
    ("L96_sym_snr20_w1234", 300, 400, 260, 96, "sym", "f64", "f64", "snr", 20.0, (1, 2, 3, 4), 2, 0, 0),
    ("L96_asym_snr20_w1234", 300, 400, 260, 96, "asym", "f64", "f64", "snr", 20.0, (1, 2, 3, 4), 2, 0, 0),
    ("L96_asym_snr35_w1234_tab", 150, 200, 90, 96, "asym", "f64", "f64", "snr", 35.0, (1, 2, 3, 4), 2, 1, 1),
    ("L96_sym_f32_in_w1234_ta", 190, 330, 170, 96, "sym", "f32", "f64", "snr", 25.0, (1, 2, 3, 4), 2, 1, 0),
    ("L96_target_w4", 192, 288, 200, 96, "asym", "f64", "f64", "target", 10.0, (1, 4), 4, 0, 0),
]


def _inputs(M, K, N, dt, ta, tb, seed):
    r = np.random.default_rng(seed)
    A = r.standard_normal((M, K)) * (1.0 + 9.0 * r.random((M, 1)))      # uneven row scales
    B = r.laplace(0.0, 1.0, (K, N))
    if M >= 64 and K >= 64:
        A[:64, :64] = 0.0                                                 # an all-zero block
    A = A.astype(dt)
    B = B.astype(dt)
    At = to_dev(A.T.copy()).t() if ta else to_dev(A)
    Bt = to_dev(B.T.copy()).t() if tb else to_dev(B)
    return A, B, At, Bt


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_stagewise_parity(td, case):
    name, M, K, N, L, form, ind, prec, ctrl, snr, wal, fw, ta, tb = case
    log(f"[parity] {name}: M={M} K={K} N={N} L={L} {form} in={ind} prec={prec} ctrl={ctrl} snr={snr}")
    dt = np.float64 if ind == "f64" else np.float32
    A, B, Ad, Bd = _inputs(M, K, N, dt, ta, tb, seed=zlib.crc32(name.encode()))
    rmax = float(2 ** 20) if L == 64 else float(2 ** 21)
    if fw == 3:
        rmax = float(2 ** 14)            # three 16-bit slots: inside the FP64 mantissa
    if fw == 4:
        rmax = float(2 ** 9)             # four 12-bit slots
    calib, tabs = device_calib(td, L, form, prec, tuple(w for w in wal if w > 1) or (2,))
    cfg = oracle_cfg(L, form, prec, ctrl, snr, wal, fw, rmax, 127.0)
    res = pl.run(A, B, cfg, calib=tabs, keep=True)

    desc = td.make_desc(Ad, Bd, L=L, form=form, prec=prec, ctrl=ctrl, snr_db=snr, w_allowed=wal,
                        fixed_w=fw, fixed_rmax=rmax, sep_q=127.0)
    plan = td.tdgemm_plan(desc, Ad, Bd, calib if ctrl in ("snr", "target") else None)
    sa, sb, pairs, budget = td.tdgemm_plan_export(plan)
    nI, nL, nJ, npairs = plan.dims
    tiles = [(i, j) for i in range(nI) for j in range(nJ)]
    compare_plan(pairs, budget, sa, sb, res, tiles)

    pt = td.torch_dtype(desc.prec)
    n = td.slot_elems(plan)
    bufs = {k: torch.full((n,), float("nan"), dtype=pt, device="cuda") for k in
            ("qA", "qB", "pA", "pB", "R", "r")}
    C_st = torch.full((M, N), float("nan"), dtype=pt, device="cuda")
    C_fu = torch.full((M, N), float("nan"), dtype=pt, device="cuda")
    td.tdgemm_compand(plan, Ad, Bd, bufs["qA"], bufs["qB"])
    td.tdgemm_pack(plan, bufs["qA"], bufs["qB"], bufs["pA"], bufs["pB"])
    td.tdgemm_gemm(plan, bufs["pA"], bufs["pB"], bufs["R"], fused=0)
    td.tdgemm_unpack(plan, bufs["R"], bufs["r"], C_st)
    td.tdgemm_gemm(plan, Ad, Bd, C_fu, fused=1)
    torch.cuda.synchronize()
    h = {k: v.cpu().numpy().reshape(npairs, L, L) for k, v in bufs.items()}

    for i in range(nI):
        for j in range(nJ):
            for l in range(nL):
                p = (i * nJ + j) * nL + l
                tr = res.traces[(i, j, l)]
                W = int(pairs[i, j, l]["w"])
                sym = form == "sym" or W == 1
                np.testing.assert_array_equal(h["qA"][p], tr.qa, err_msg=f"qA {p}")
                np.testing.assert_array_equal(h["qB"][p], tr.qb, err_msg=f"qB {p}")
                pa = h["pA"][p].ravel()[:tr.abar.size].reshape(tr.abar.shape)
                pb = h["pB"][p].ravel()[:tr.bbar.size].reshape(tr.bbar.shape)
                np.testing.assert_array_equal(pa, tr.abar, err_msg=f"pA {p}")
                np.testing.assert_array_equal(pb, tr.bbar, err_msg=f"pB {p}")
                rows = L if sym else L // W
                np.testing.assert_array_equal(h["R"][p][:rows], tr.rbar, err_msg=f"Rbar {p}")
                np.testing.assert_array_equal(h["r"][p], tr.r, err_msg=f"r {p}")
    Cs = C_st.cpu().numpy()
    Cf = C_fu.cpu().numpy()
    assert np.all(np.isfinite(Cs)) and np.all(np.isfinite(Cf))
    np.testing.assert_array_equal(Cf, Cs)                 # fused == staged, bit for bit
    np.testing.assert_array_equal(Cs, res.C, err_msg="C vs oracle")
    assert rel_err(Cs, res.C) <= TOL[prec]
    exact_c = np.array_equal(Cs, res.C)
    ref = A.astype(np.float64) @ B.astype(np.float64)
    log(f"[parity] {name}: C rel err {rel_err(Cs, res.C):.3e} (bit-exact: {exact_c}), "
        f"SNR vs FP64 {pl.snr_db(Cs, ref):.2f} dB, W hist "
        f"{ {w: int((pairs['w'] == w).sum()) for w in (1, 2, 3, 4)} }")


DET_CASES = [
    # name, M, K, N, L, form, S, k_split, calibration (std, or W = 4 cheaper than W = 2:
    # the step-by-step greedy of the pruning)
    ("laplace512_L64", 512, 512, 512, 64, "sym", 40.0, 1, "std"),
    ("split3_L128_asym", 260, 128 * 11 + 40, 200, 128, "asym", 30.0, 3, "std"),
    ("greedy_nonmono", 192, 640, 128, 64, "sym", 86.0, 1, "scaled_w4"),
]


@pytest.mark.parametrize("case", DET_CASES, ids=[c[0] for c in DET_CASES])
def test_fused_deterministic(td, case):
    """Ten runs of plan + fused product give the same records and C bit for bit."""
    from oracle import control as ct
    from tests.oracle_tables import tables
    name, M, K, N, L, form, snr, ks, ckind = case
    log(f"[determinism] {name}: 10 runs")
    r = np.random.default_rng(zlib.crc32(name.encode()))
    A, B = r.laplace(0.0, 1.0, (M, K)), r.standard_normal((K, N))
    Ad, Bd = to_dev(A), to_dev(B)
    tabs = tables(L, form, "f64", (2, 4))
    if ckind == "scaled_w4":
        tabs = {2: tabs[2], 4: ct.CalibTable(tabs[2].r.copy(), tabs[2].s * 0.25)}
    calib = td.DeviceCalib(tabs[2].r, {W: tabs[W].s for W in (2, 4)})
    outs = []
    for _ in range(10):
        C, plan = td.matmul(Ad, Bd, calib, L=L, form=form, ctrl="snr", snr_db=snr, w_allowed=(1, 2, 4),
                            k_split=ks)
        torch.cuda.synchronize()
        outs.append((td.tdgemm_plan_export(plan)[2].tobytes(), C.cpu().numpy().tobytes()))
    assert all(o == outs[0] for o in outs[1:])


@pytest.mark.parametrize("M,K,N", [(0, 64, 64), (64, 0, 64), (64, 64, 0), (0, 0, 0)])
def test_empty_shapes(td, M, K, N):
    Ad = torch.randn(M, K, dtype=torch.float64, device="cuda")
    Bd = torch.randn(K, N, dtype=torch.float64, device="cuda")
    calib, _ = device_calib(td, 64, "sym", "f64")
    C = torch.full((M, N), float("nan"), dtype=torch.float64, device="cuda")
    td.matmul(Ad, Bd, calib, out=C, L=64)
    torch.cuda.synchronize()
    assert torch.all(C == 0)                              # K = 0 gives zeros; others are empty


@pytest.mark.parametrize("form,prec,W,L", [("sym", "f64", 2, 64), ("asym", "f64", 2, 64),
                                           ("sym", "f64", 4, 64), ("sym", "f32", 2, 64),
                                           ("asym", "f64", 2, 128), ("sym", "f64", 3, 96),
                                           ("asym", "f64", 3, 96), ("asym", "f64", 2, 96),
                                           ("sym", "f64", 4, 96), ("asym", "f64", 4, 96)])
def test_calibration_parity(td, form, prec, W, L):
    """Sec. 4.B measurement on the GPU path equals the oracle's on the same draws."""
    from oracle import calibration as cal
    ua, ub = workloads.calib_uniforms(L)
    qs = [q for q in cal.q_grid(1 << 18 if prec == "f64" else 1 << 10)][::3]
    r, m, s = td.tdgemm_calibrate(L, W, form, prec, qs, to_dev(ua), to_dev(ub))
    for t, q in enumerate(qs):
        R, mo, so = cal.measure(L, W, form, prec, q, ua, ub)
        assert r[t] == R
        if math.isinf(so):
            assert math.isinf(s[t])
        else:
            assert s[t] == so and m[t] == mo, (q, s[t], so, m[t], mo)
    log(f"[calib] {form} {prec} W={W} L={L}: {len(qs)} points equal; first nonzero s at R="
        f"{next((x for x, y in zip(r, s) if y > 0), None)}")


SPLIT_CASES = [
    # name, M, K, N, L, form, prec, k_split, ta, tb
    ("split3_sym_L64", 130, 64 * 11 + 5, 150, 64, "sym", "f64", 3, 0, 0),
    ("split4_asym_L128_ta", 200, 128 * 9, 70, 128, "asym", "f64", 4, 1, 0),
    ("split5_sym_L96_f32", 96, 96 * 13 + 40, 100, 96, "sym", "f32", 5, 0, 1),
    ("split_all_asym_L96", 100, 96 * 6, 96, 96, "asym", "f64", 64, 0, 0),
]


# Shapes whose tiles fill the last round of an XCD (one tile per CU at L = 96 and
# 128, two at L = 64) at least half: the fused launch runs each XCD's border
# tiles last. Ragged M and N, so there are border tiles on both edges.
ORDER_CASES = [
    # name, M, K, N, L, form; tiles per XCD (ceil(tiles / 8)) and its last round
    ("order_L64_256tiles", 1014, 128, 1014, 64, "sym"),      # 256 tiles: 32 per XCD, 32 of 64
    ("order_L128_121tiles", 1388, 256, 1388, 128, "sym"),    # 121 tiles: 16 per XCD, 16 of 32
    ("order_L96_121tiles", 1026, 192, 1026, 96, "asym"),     # 121 tiles: 16 per XCD, 16 of 32
    ("order_L128_row_order", 1100, 256, 1300, 128, "sym"),   # 99 tiles: 13 per XCD, row order
]


@pytest.mark.parametrize("case", ORDER_CASES, ids=[c[0] for c in ORDER_CASES])
def test_fused_tile_order_parity(td, case):
    """The fused kernel's tile order (border tiles last in each XCD's share, or
    the row order) covers every tile once: C equals the staged path and the
    oracle bit for bit."""
    name, M, K, N, L, form = case
    log(f"[order] {name}: M={M} K={K} N={N} L={L} {form}")
    A, B, Ad, Bd = _inputs(M, K, N, np.float64, 0, 0, seed=zlib.crc32(name.encode()))
    wal = (1, 2, 3) if L == 96 else (1, 2, 4)
    calib, tabs = device_calib(td, L, form, "f64", tuple(w for w in wal if w > 1))
    cfg = oracle_cfg(L, form, "f64", "snr", 30.0, wal, 2, 0.0, 127.0)
    res = pl.run(A, B, cfg, calib=tabs)
    desc = td.make_desc(Ad, Bd, L=L, form=form, prec="f64", ctrl="snr", snr_db=30.0, w_allowed=wal)
    plan = td.tdgemm_plan(desc, Ad, Bd, calib)
    C_fu = torch.full((M, N), float("nan"), dtype=torch.float64, device="cuda")
    td.tdgemm_gemm(plan, Ad, Bd, C_fu, fused=1)
    n = td.slot_elems(plan)
    bufs = {k: torch.full((n,), float("nan"), dtype=torch.float64, device="cuda") for k in
            ("qA", "qB", "pA", "pB", "R", "r")}
    C_st = torch.full((M, N), float("nan"), dtype=torch.float64, device="cuda")
    td.tdgemm_compand(plan, Ad, Bd, bufs["qA"], bufs["qB"])
    td.tdgemm_pack(plan, bufs["qA"], bufs["qB"], bufs["pA"], bufs["pB"])
    td.tdgemm_gemm(plan, bufs["pA"], bufs["pB"], bufs["R"], fused=0)
    td.tdgemm_unpack(plan, bufs["R"], bufs["r"], C_st)
    torch.cuda.synchronize()
    Cf, Cs = C_fu.cpu().numpy(), C_st.cpu().numpy()
    assert np.all(np.isfinite(Cf))
    np.testing.assert_array_equal(Cf, Cs)
    np.testing.assert_array_equal(Cf, res.C, err_msg="C vs oracle")
    nI, nL, nJ, _ = plan.dims
    log(f"[order] {name}: {nI * nJ} tiles, C bit-exact against the staged path and the oracle")

@pytest.mark.parametrize("case", SPLIT_CASES, ids=[c[0] for c in SPLIT_CASES])
def test_k_split_parity(td, case):
    """The l-sum of eq. (2) in groups of consecutive subblocks (k_split): the fused
    kernel with one workgroup per group plus the ordered group sum equals the staged
    path bit for bit, and the oracle with the same grouping within the stated bound."""
    name, M, K, N, L, form, prec, ks, ta, tb = case
    log(f"[split] {name}: M={M} K={K} N={N} L={L} {form} {prec} k_split={ks}")
    dt = np.float64 if prec == "f64" else np.float32
    A, B, Ad, Bd = _inputs(M, K, N, dt, ta, tb, seed=zlib.crc32(name.encode()))
    wal = (1, 2, 3) if L == 96 else (1, 2, 4)
    if prec == "f32":
        wal = (1, 2)
    snr = 40.0 if prec == "f64" else 15.0
    calib, tabs = device_calib(td, L, form, prec, tuple(w for w in wal if w > 1))
    cfg = oracle_cfg(L, form, prec, "snr", snr, wal, 2, 1.0, 127.0)
    import dataclasses
    ref = pl.run(A, B, dataclasses.replace(cfg, k_groups=ks), calib=tabs)
    desc = td.make_desc(Ad, Bd, L=L, form=form, prec=prec, ctrl="snr", snr_db=snr, w_allowed=wal,
                        k_split=ks)
    plan = td.tdgemm_plan(desc, Ad, Bd, calib)
    pt = td.torch_dtype(desc.prec)
    n = td.slot_elems(plan)
    bufs = {k: torch.empty((n,), dtype=pt, device="cuda") for k in ("qA", "qB", "pA", "pB", "R")}
    C_st = torch.full((M, N), float("nan"), dtype=pt, device="cuda")
    C_fu = torch.full((M, N), float("nan"), dtype=pt, device="cuda")
    td.tdgemm_compand(plan, Ad, Bd, bufs["qA"], bufs["qB"])
    td.tdgemm_pack(plan, bufs["qA"], bufs["qB"], bufs["pA"], bufs["pB"])
    td.tdgemm_gemm(plan, bufs["pA"], bufs["pB"], bufs["R"], fused=0)
    td.tdgemm_unpack(plan, bufs["R"], None, C_st)
    td.tdgemm_gemm(plan, Ad, Bd, C_fu, fused=1)
    torch.cuda.synchronize()
    Cs, Cf = C_st.cpu().numpy(), C_fu.cpu().numpy()
    assert np.all(np.isfinite(Cf))
    np.testing.assert_array_equal(Cf, Cs)
    np.testing.assert_array_equal(Cf, ref.C, err_msg="C vs the oracle's grouping")
    # eq. (2) as one ascending sum: the grouping changes roundings only
    plain = pl.run(A, B, cfg, calib=tabs).C
    assert_elementwise(Cf, plain, A, B, TOL[prec], "C vs the ascending l-sum")
    assert rel_err(Cf, plain) <= TOL[prec]
    log(f"[split] {name}: C rel err vs the ascending sum {rel_err(Cf, plain):.3e}")


def test_calibration_table_cache(td, tmp_path, monkeypatch):
    """A table measured on the GPU and stored is read back bit for bit, without measuring."""
    from paper_1110_5765_amd import calib
    p = str(tmp_path / "calib_L64_sym_f64.json")
    _, r, table = calib.device_table(64, "sym", "f64", (2, 4), cache=p)

    def no_measure(*a, **k):
        raise AssertionError("measured although a matching table is stored")

    monkeypatch.setattr(calib.td, "tdgemm_calibrate", no_measure)
    dev, r2, t2 = calib.device_table(64, "sym", "f64", (2, 4), cache=p)
    assert np.asarray(r2).tobytes() == np.asarray(r, dtype=np.float64).tobytes()
    for W in (2, 4):
        assert t2[W].tobytes() == np.asarray(table[W], dtype=np.float64).tobytes()
    s = dev.s.cpu().numpy().reshape(3, -1)
    assert s[0].tobytes() == t2[2].tobytes() and s[2].tobytes() == t2[4].tobytes()


LDC_CASES = [
    # name, M, K, N, L, form, in/pack precision, k_split
    ("ldc_sym_L64", 130, 200, 150, 64, "sym", "f64", 1),
    ("ldc_asym_L128_split3", 200, 128 * 5, 70, 128, "asym", "f64", 3),
    ("ldc_sym_L96_f32", 100, 250, 90, 96, "sym", "f32", 1),
]


@pytest.mark.parametrize("case", LDC_CASES, ids=[c[0] for c in LDC_CASES])
def test_ldc_wider_than_n(td, case):
    """C written with a leading dimension above N: the M x N part equals the
    ldc = N result bit for bit (fused and staged), the padding stays untouched."""
    name, M, K, N, L, form, prec, ks = case
    log(f"[parity] {name}: M={M} K={K} N={N} L={L} {form} {prec} k_split={ks}, ldc={N + 37}")
    dt = np.float64 if prec == "f64" else np.float32
    A, B, Ad, Bd = _inputs(M, K, N, dt, 0, 0, seed=zlib.crc32(name.encode()))
    wal = (1, 2) if prec == "f32" else ((1, 2, 3) if L == 96 else (1, 2, 4))
    calib, _ = device_calib(td, L, form, prec, tuple(w for w in wal if w > 1))
    snr = 30.0 if prec == "f64" else 12.0
    pt = torch.float64 if prec == "f64" else torch.float32
    ldc = N + 37
    d0 = td.make_desc(Ad, Bd, L=L, form=form, prec=prec, ctrl="snr", snr_db=snr, w_allowed=wal, k_split=ks)
    d1 = td.make_desc(Ad, Bd, L=L, form=form, prec=prec, ctrl="snr", snr_db=snr, w_allowed=wal, k_split=ks,
                      ldc=ldc)
    p0 = td.tdgemm_plan(d0, Ad, Bd, calib)
    p1 = td.tdgemm_plan(d1, Ad, Bd, calib)
    C0 = torch.full((M, N), float("nan"), dtype=pt, device="cuda")
    C1 = torch.full((M, ldc), 12345.0, dtype=pt, device="cuda")
    C2 = torch.full((M, ldc), -777.0, dtype=pt, device="cuda")
    td.tdgemm_gemm(p0, Ad, Bd, C0, fused=1)
    td.tdgemm_gemm(p1, Ad, Bd, C1, fused=1)
    n = td.slot_elems(p1)
    bufs = [torch.empty(n, dtype=pt, device="cuda") for _ in range(5)]
    td.tdgemm_compand(p1, Ad, Bd, bufs[0], bufs[1])
    td.tdgemm_pack(p1, bufs[0], bufs[1], bufs[2], bufs[3])
    td.tdgemm_gemm(p1, bufs[2], bufs[3], bufs[4], fused=0)
    td.tdgemm_unpack(p1, bufs[4], None, C2)
    torch.cuda.synchronize()
    c0, c1, c2 = C0.cpu().numpy(), C1.cpu().numpy(), C2.cpu().numpy()
    assert np.all(np.isfinite(c0))
    assert c1[:, :N].tobytes() == np.ascontiguousarray(c0).tobytes()
    assert c2[:, :N].tobytes() == np.ascontiguousarray(c0).tobytes()
    assert np.all(c1[:, N:] == 12345.0) and np.all(c2[:, N:] == -777.0)


@pytest.mark.parametrize("form,L,ta,tb", [("sym", 64, 0, 0), ("asym", 128, 1, 0), ("sym", 96, 0, 1)])
def test_padded_operands(td, form, L, ta, tb):
    """A and B as slices of wider matrices (lda, ldb above the stored row length):
    plan and C equal those of contiguous copies bit for bit."""
    M, K, N = 150, 260, 110
    log(f"[parity] padded operands: {form} L={L} ta={ta} tb={tb}")
    rng = np.random.default_rng(L + 7 * ta + 13 * tb)
    A = rng.standard_normal((M, K))
    B = rng.laplace(0.0, 1.0, (K, N))

    def padded(X, t):
        if t:   # stored transposed, K x M (or N x K) rows padded by 9
            big = torch.full((X.shape[1], X.shape[0] + 9), float("nan"), dtype=torch.float64, device="cuda")
            big[:, :X.shape[0]] = to_dev(X.T.copy())
            return big[:, :X.shape[0]].t()
        big = torch.full((X.shape[0], X.shape[1] + 5), float("nan"), dtype=torch.float64, device="cuda")
        big[:, :X.shape[1]] = to_dev(X)
        return big[:, :X.shape[1]]

    Ap, Bp = padded(A, ta), padded(B, tb)
    Ac, Bc = to_dev(A), to_dev(B)
    wal = (1, 2, 3) if L == 96 else (1, 2, 4)
    calib, _ = device_calib(td, L, form, "f64", tuple(w for w in wal if w > 1))
    outs = []
    for a, b in ((Ac, Bc), (Ap, Bp)):
        d = td.make_desc(a, b, L=L, form=form, ctrl="snr", snr_db=30.0, w_allowed=wal)
        p = td.tdgemm_plan(d, a, b, calib)
        C = torch.full((M, N), float("nan"), dtype=torch.float64, device="cuda")
        td.tdgemm_gemm(p, a, b, C, fused=1)
        torch.cuda.synchronize()
        outs.append((td.tdgemm_plan_export(p)[2], C.cpu().numpy()))
    assert outs[0][0].tobytes() == outs[1][0].tobytes()
    assert np.all(np.isfinite(outs[0][1])) and outs[0][1].tobytes() == outs[1][1].tobytes()
