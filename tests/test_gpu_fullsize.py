"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times, on sampled outputs the oracle computes one inner kernel at a
time.

* 4096^3 sweep point (Gaussian and Laplace inputs, L = 128 and 64): the plan
  (statistics of every block; pair records and budgets of the sampled inner
  kernels) bit-exact, and every sampled L x L tile of the fused product within
  1e-12 (relative, Frobenius) of the oracle's. Over the whole output, the SNR
  against the FP64 product is logged and must be finite.
* 8192^3 block-scaled INT8 / FP8: for sampled tiles the byte operands of their
  panels bit-exact and C bit-exact (INT8) or within the FP8 bound (see the
  block-scaled parity tests). A tile of the block-scaled product depends only on
  the blocks of its A row panel and B column panel, so the oracle runs on those
  two panels.
Sampled tiles: the four corners and four seeded draws."""
import math

import numpy as np
import pytest

import workloads
from oracle import pipeline as pl
from oracle import precision as pr
from tests.gpu_common import compare_plan, device_calib, log, oracle_cfg, rel_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def td():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1110_5765_amd import tdgemm
    return tdgemm


def _sample_tiles(nI, nJ, seed, extra=4):
    r = np.random.default_rng(seed)
    tiles = {(0, 0), (0, nJ - 1), (nI - 1, 0), (nI - 1, nJ - 1)}
    while len(tiles) < 4 + extra:
        tiles.add((int(r.integers(nI)), int(r.integers(nJ))))
    return sorted(tiles)


SWEEP_CASES = [
    # name, distribution, L, form, S (dB), allowed W
    ("gauss_L128_sym_S40", "gaussian", 128, "sym", 40.0, (1, 2, 4)),
    ("laplace_L128_sym_S20", "laplace", 128, "sym", 20.0, (1, 2, 4)),
    ("gauss_L64_asym_S28", "gaussian", 64, "asym", 28.0, (1, 2, 4)),
]


@pytest.mark.parametrize("case", SWEEP_CASES, ids=[c[0] for c in SWEEP_CASES])
def test_sweep_full_size_sampled(td, case):
    name, dist, L, form, snr, wal = case
    n = 4096
    log(f"[fullsize] {name}: {n}^3 {dist}, L={L}, {form}, S={snr} dB, W={wal}")
    A, B = workloads.sweep(dist, n=n)
    Ad, Bd = to_dev(A), to_dev(B)
    calib, tabs = device_calib(td, L, form, "f64", tuple(w for w in wal if w > 1))
    desc = td.make_desc(Ad, Bd, L=L, form=form, ctrl="snr", snr_db=snr, w_allowed=wal)
    ws = torch.empty(td.tdgemm_workspace_size(desc), dtype=torch.uint8, device="cuda")
    C = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda")
    plan = td.tdgemm_plan(desc, Ad, Bd, calib, ws)
    td.tdgemm_gemm(plan, Ad, Bd, C, fused=1)
    torch.cuda.synchronize()
    sa, sb, pairs, budget = td.tdgemm_plan_export(plan)
    nI, nL, nJ, _ = plan.dims

    tiles = _sample_tiles(nI, nJ, seed=len(name))
    cfg = oracle_cfg(L, form, "f64", "snr", snr, wal, 2, 0.0, 127.0)
    oplan = pl.make_plan(A, B, cfg, tabs, tiles=tiles)
    res = pl.run(A, B, cfg, tabs, tiles=tiles, plan=oplan)
    compare_plan(pairs, budget, sa, sb, res, tiles)

    Ch = C.cpu().numpy()
    assert np.all(np.isfinite(Ch))
    exact = 0
    for (i, j) in tiles:
        got = Ch[i * L:(i + 1) * L, j * L:(j + 1) * L]
        want = res.C[i * L:(i + 1) * L, j * L:(j + 1) * L]
        err = rel_err(got, want)
        assert err <= 1e-12, (i, j, err)
        exact += int(np.array_equal(got, want))
    ref = torch.matmul(Ad, Bd)
    e2 = float(torch.sum((C - ref) ** 2))
    snr_out = 10.0 * math.log10(float(torch.sum(ref * ref)) / e2) if e2 > 0 else math.inf
    assert math.isfinite(snr_out) or e2 == 0.0
    hist = {w: int((pairs["w"] == w).sum()) for w in (1, 2, 4)}
    log(f"[fullsize] {name}: {len(tiles)} tiles within 1e-12 ({exact} bit-exact), "
        f"SNR vs FP64 {snr_out:.2f} dB, W hist {hist}")


@pytest.mark.parametrize("fmt,q", [("i8", 127.0), ("e4m3", 448.0)])
def test_block_scaled_full_size_sampled(td, fmt, q):
    n, L = 8192, 128
    log(f"[fullsize] block-scaled {fmt}: {n}^3 Laplace, Q={q}")
    A, B = workloads.precision(n)
    Ad, Bd = to_dev(A), to_dev(B)
    desc = td.make_desc(Ad, Bd, L=L, prec=fmt, ctrl="separable", fixed_w=1, sep_q=q)
    ws = torch.empty(td.tdgemm_workspace_size(desc), dtype=torch.uint8, device="cuda")
    plan = td.tdgemm_plan(desc, Ad, Bd, None, ws)
    sh = td.block_scaled_shapes(plan)
    qA = torch.empty(sh["qA"], dtype=torch.uint8, device="cuda")
    qB = torch.empty(sh["qB"], dtype=torch.uint8, device="cuda")
    C = torch.full((n, n), float("nan"), dtype=torch.float32, device="cuda")
    td.tdgemm_compand(plan, Ad, Bd, qA, qB)
    td.tdgemm_gemm(plan, qA, qB, C, fused=1)
    torch.cuda.synchronize()
    nb = n // L
    tiles = _sample_tiles(nb, nb, seed=7 if fmt == "i8" else 8)
    Ch = C.cpu().numpy()
    assert np.all(np.isfinite(Ch))
    qa_all = qA.cpu().numpy()
    qb_all = qB.cpu().numpy()
    for (i, j) in tiles:
        a = A[i * L:(i + 1) * L, :]
        b = B[:, j * L:(j + 1) * L]
        ref = pr.run(a, b, L, fmt, q, keep_products=False)
        np.testing.assert_array_equal(qa_all[i * L:(i + 1) * L, :], pr.codes(ref.qa, fmt))
        np.testing.assert_array_equal(qb_all[j * L:(j + 1) * L, :], pr.codes(ref.qb, fmt).T)
        got = Ch[i * L:(i + 1) * L, j * L:(j + 1) * L]
        if fmt == "i8":
            np.testing.assert_array_equal(got, ref.C, err_msg=f"tile {(i, j)}")
        else:
            assert rel_err(got, ref.C) <= 1e-4, (i, j, rel_err(got, ref.C))
    ref_all = torch.matmul(Ad, Bd)
    e2 = float(torch.sum((C.double() - ref_all) ** 2))
    snr_out = 10.0 * math.log10(float(torch.sum(ref_all * ref_all)) / e2)
    log(f"[fullsize] block-scaled {fmt}: {len(tiles)} tiles match the oracle, SNR vs FP64 {snr_out:.2f} dB")
