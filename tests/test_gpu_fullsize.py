"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times, on sampled outputs the oracle computes one inner kernel at a
time.

* 4096^3 sweep point (Gaussian and Laplace inputs, L = 128 and 64): the plan
  (statistics of every block; pair records and budgets of the sampled inner
  kernels) bit-exact, and every sampled L x L tile of the fused product equal
  to the oracle's element by element. Over the whole output, the SNR against
  the FP64 product must reach the target less 1 dB (the budget bounds the
  expected noise of every inner kernel).
* The scatter workload (X 2000 x 10304 float32): X^T X (10304^2, K = 2000,
  A transposed, FP64 packing, an 80-column K tail at L = 128) on sampled tiles,
  and X P (P 10304 x 200, grouped l-sum as the benchmark runs it) in full.
* The perceptron's packed products of one training step at batch 4096 (FP32
  packing, L = 128, S = 20 dB, the benchmark's settings): forward, input
  gradient and weight gradient of the 1024 -> 1024 layer and forward and
  weight gradient of the 512 -> 1024 layer, on sampled tiles.
* 2D-PCA on the synthetic 288 x 288 images: G over the 75 stacked training
  images (K = 21600, L = 96, grouped l-sum) and the projections, in full.
  Grouped l-sums equal the oracle with the same grouping bit for bit, and the
  plain ascending sum within 1e-12 (FP64) / 1e-5 (FP32) of |A||B|.
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
from tests.gpu_common import assert_elementwise, compare_plan, device_calib, log, oracle_cfg, rel_err, to_dev

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
    for (i, j) in tiles:
        got = Ch[i * L:(i + 1) * L, j * L:(j + 1) * L]
        want = res.C[i * L:(i + 1) * L, j * L:(j + 1) * L]
        np.testing.assert_array_equal(got, want, err_msg=f"tile {(i, j)}")
        assert rel_err(got, want) <= 1e-12
    ref = torch.matmul(Ad, Bd)
    e2 = float(torch.sum((C - ref) ** 2))
    snr_out = 10.0 * math.log10(float(torch.sum(ref * ref)) / e2) if e2 > 0 else math.inf
    hist = {w: int((pairs["w"] == w).sum()) for w in (1, 2, 4)}
    log(f"[fullsize] {name}: {len(tiles)} tiles bit-exact, SNR vs FP64 {snr_out:.2f} dB "
        f"(target {snr:g}, margin {snr_out - snr:+.2f} dB), W hist {hist}")
    assert snr_out >= snr - 1.0, (snr_out, snr)


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


def _tile_blocks(C, tiles, L):
    return {(i, j): C[i * L:(i + 1) * L, j * L:(j + 1) * L] for (i, j) in tiles}


def _check_product(td, name, A, B, Ad, Bd, C_dev, cfg, tabs, tiles, ks, tol):
    """C_dev against the oracle on the given inner kernels (all when tiles is None):
    bit for bit with the library's grouping of the l-sum, and within tol x |A||B|
    element by element of the plain ascending sum."""
    import dataclasses
    L = cfg.L
    M, N = C_dev.shape
    Ch = C_dev.cpu().numpy()
    assert np.all(np.isfinite(Ch))
    grouped = pl.run(A, B, dataclasses.replace(cfg, k_groups=ks), tabs, tiles=tiles).C
    plain = grouped if ks == 1 else pl.run(A, B, cfg, tabs, tiles=tiles).C
    if tiles is None:
        np.testing.assert_array_equal(Ch, grouped, err_msg=name)
        assert_elementwise(Ch, plain, A, B, tol, name)
        log(f"[fullsize] {name}: all of C bit-exact with k_split {ks}; rel err vs the ascending "
            f"sum {rel_err(Ch, plain):.2e}")
        return
    for (i, j) in tiles:
        r0, c0 = i * L, j * L
        got = Ch[r0:r0 + L, c0:c0 + L]
        np.testing.assert_array_equal(got, grouped[r0:r0 + L, c0:c0 + L], err_msg=f"{name} tile {(i, j)}")
        assert_elementwise(got, plain[r0:r0 + L, c0:c0 + L], A[r0:r0 + L, :], B[:, c0:c0 + L], tol,
                           f"{name} tile {(i, j)}")
    log(f"[fullsize] {name}: {len(tiles)} sampled tiles bit-exact with k_split {ks}")


def test_scatter_full_size(td):
    """X^T X and X P of the scatter workload, as the benchmark runs them (S = 40 dB)."""
    L, snr, wal = 128, 40.0, (1, 2, 4)
    xs, ps = workloads.scatter()
    log(f"[fullsize] scatter: X {xs.shape}, P {ps.shape}, L={L}, S={snr}")
    X, P = to_dev(xs), to_dev(ps)
    calib, tabs = device_calib(td, L, "sym", "f64", (2, 4))
    cfg = oracle_cfg(L, "sym", "f64", "snr", snr, wal, 2, 0.0, 127.0)
    for name, (A, B, Ad, Bd) in {"XtX": (xs.T, xs, X.t(), X), "XP": (xs, ps, X, P)}.items():
        M, K = A.shape
        N = B.shape[1]
        ks = td.auto_k_split(M, N, K, L, "f64")
        desc = td.make_desc(Ad, Bd, L=L, form="sym", prec="f64", ctrl="snr", snr_db=snr, w_allowed=wal,
                            k_split=ks)
        plan = td.tdgemm_plan(desc, Ad, Bd, calib)
        C = torch.empty((M, N), dtype=torch.float64, device="cuda")
        td.tdgemm_gemm(plan, Ad, Bd, C, fused=1)
        torch.cuda.synchronize()
        nI, nL, nJ, _ = plan.dims
        tiles = _sample_tiles(nI, nJ, seed=M) if nI * nJ > 64 else None
        A64, B64 = A.astype(np.float64), B.astype(np.float64)
        _check_product(td, f"scatter {name} {M}x{K}x{N}", A64, B64, Ad, Bd, C, cfg, tabs, tiles, ks, 1e-12)


def test_perceptron_step_products_full_size(td):
    """One training step's packed products at batch 4096 with the benchmark's settings."""
    from paper_1110_5765_amd import autograd
    L, snr = 128, 20.0
    Ws, _, xs, _ = workloads.mlp()
    rng = np.random.default_rng(4096)
    X = xs[0]                                                        # 4096 x 512
    H = np.maximum(rng.standard_normal((4096, 1024)), 0.0).astype(np.float32)
    G2 = (rng.standard_normal((4096, 1024)) * 1e-3).astype(np.float32)
    G1 = (rng.standard_normal((4096, 1024)) * 1e-3).astype(np.float32)
    calib, tabs = device_calib(td, L, "sym", "f32", (2,))
    tdc = autograd.TDContext(autograd.TDConfig(L=L, form="sym", prec="f32", ctrl="snr", snr_db=snr,
                                               w_allowed=(1, 2), min_dim=2 * L), calib)
    cfg = oracle_cfg(L, "sym", "f32", "snr", snr, (1, 2), 2, 0.0, 127.0)
    Xd, Hd, G2d, G1d = to_dev(X), to_dev(H), to_dev(G2), to_dev(G1)
    W1d, W2d = to_dev(Ws[0]), to_dev(Ws[1])
    products = {
        "layer2 Y = H W2": (H, Ws[1], Hd, W2d),
        "layer2 dX = dY W2^T": (G2, Ws[1].T, G2d, W2d.t()),
        "layer2 dW = H^T dY": (H.T, G2, Hd.t(), G2d),
        "layer1 Y = X W1": (X, Ws[0], Xd, W1d),
        "layer1 dW = X^T dY": (X.T, G1, Xd.t(), G1d),
    }
    for name, (A, B, Ad, Bd) in products.items():
        M, K = A.shape
        N = B.shape[1]
        log(f"[fullsize] perceptron {name}: {M}x{K} by {K}x{N}")
        C = tdc.matmul(Ad, Bd)
        torch.cuda.synchronize()
        assert tdc.plain_calls == 0
        ks = td.auto_k_split(M, N, K, L, "f32")
        nI, nJ = -(-M // L), -(-N // L)
        tiles = _sample_tiles(nI, nJ, seed=M + N)
        _check_product(td, f"perceptron {name}", np.ascontiguousarray(A), np.ascontiguousarray(B), Ad, Bd,
                       C, cfg, tabs, tiles, ks, 1e-5)


def test_pca2d_full_size(td):
    """G over the 75 stacked 288 x 288 training images and the projections of the
    training and test images onto 10 axes, as the benchmark runs them (S = 30 dB)."""
    L, snr, d, size = 96, 30.0, 10, 288
    tr, _, te, _ = workloads.faces()
    mu = tr.mean(0)
    S = (tr - mu).reshape(-1, size).astype(np.float32)
    T = (te - mu).reshape(-1, size).astype(np.float32)
    log(f"[fullsize] 2D-PCA: S {S.shape}, T {T.shape}, L={L}, S={snr}")
    calib, tabs = device_calib(td, L, "sym", "f32", (2,))
    cfg = oracle_cfg(L, "sym", "f32", "snr", snr, (1, 2), 2, 0.0, 127.0)
    Sd, Td = to_dev(S), to_dev(T)

    def lib(Ad, Bd):
        M, K = Ad.shape
        N = Bd.shape[1]
        ks = td.auto_k_split(M, N, K, L, "f32")
        desc = td.make_desc(Ad, Bd, L=L, form="sym", prec="f32", ctrl="snr", snr_db=snr, w_allowed=(1, 2),
                            k_split=ks)
        plan = td.tdgemm_plan(desc, Ad, Bd, calib)
        C = torch.empty((M, N), dtype=torch.float32, device="cuda")
        td.tdgemm_gemm(plan, Ad, Bd, C, fused=1)
        torch.cuda.synchronize()
        return C, ks

    G, ks = lib(Sd.t(), Sd)
    _check_product(td, "2D-PCA G = S^T S", np.ascontiguousarray(S.T), S, Sd.t(), Sd, G, cfg, tabs, None, ks, 1e-5)
    _, V = np.linalg.eigh(G.cpu().numpy().astype(np.float64))
    Xp = np.ascontiguousarray(V[:, ::-1][:, :d]).astype(np.float32)
    Xd = to_dev(Xp)
    for name, (A, Ad) in {"Y = S X": (S, Sd), "Y = T X": (T, Td)}.items():
        Y, ks = lib(Ad, Xd)
        _check_product(td, f"2D-PCA {name}", A, Xp, Ad, Xd, Y, cfg, tabs, None, ks, 1e-5)
