"""GPU parity of the INT8 / FP8 block-scaled form (C-ABI) against the oracle.

Bar: block statistics and pair records bit-exact; byte operands bit-exact;
INT8 per-pair products bit-exact (exact integers) and C bit-exact (the same
float32 operations in the same order). FP8: the matrix cores of gfx950 do not
round a 128-term sum of (exact) E4M3 products like IEEE float32 does, and the
order of their additions is not specified. The bar is the worst-case error of
a float32 sum of n = 128 terms p_k with round-to-nearest in any order,
gamma_(n-1) sum |p_k| <= 127 2^-24 128 max|p_k| < 2^-10 max|p_k|, per output;
measured, each sum is within 2^-11.2 max|p_k|. On C the bar is 1e-4 relative
(Frobenius). The output SNR against the float64 product is logged for every
case."""
import math
import zlib

import numpy as np
import pytest

from oracle import precision as pr
from tests.gpu_common import log, rel_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def td():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1110_5765_amd import tdgemm
    return tdgemm


CASES = [
    # name, M, K, N, fmt, q, in dtype, ta, tb
    ("i8_ragged", 300, 400, 260, "i8", 127.0, "f64", 0, 0),
    ("i8_q100_trans_a", 200, 260, 140, "i8", 100.0, "f64", 1, 0),
    ("i8_trans_b_f32", 130, 384, 250, "i8", 127.0, "f32", 0, 1),
    ("i8_k_below_L", 150, 40, 130, "i8", 127.0, "f64", 0, 0),
    ("e4m3_ragged", 300, 400, 260, "e4m3", 448.0, "f64", 0, 0),
    ("e4m3_q200_trans_ab", 140, 300, 200, "e4m3", 200.0, "f64", 1, 1),
    ("e4m3_f32", 256, 256, 256, "e4m3", 448.0, "f32", 0, 0),
]


def _inputs(M, K, N, dt, seed):
    r = np.random.default_rng(seed)
    A = r.laplace(0.0, 1.0, (M, K)) * (1.0 + 5.0 * r.random((M, 1)))
    B = r.standard_normal((K, N))
    if M >= 128 and K >= 128:
        A[:128, :128] = 0.0                   # an all-zero block
    if M > 1 and K > 130:
        A[1, 130] = -1e-30                    # rounds to a negative zero
    return A.astype(dt), B.astype(dt)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_block_scaled_parity(td, case):
    name, M, K, N, fmt, q, ind, ta, tb = case
    log(f"[precision] {name}: M={M} K={K} N={N} {fmt} Q={q} in={ind} ta={ta} tb={tb}")
    dt = np.float64 if ind == "f64" else np.float32
    A, B = _inputs(M, K, N, dt, zlib.crc32(name.encode()))
    ref = pr.run(A.astype(np.float64), B.astype(np.float64), 128, fmt, q)
    Ad = to_dev(A.T.copy()).t() if ta else to_dev(A)
    Bd = to_dev(B.T.copy()).t() if tb else to_dev(B)
    desc = td.make_desc(Ad, Bd, L=128, prec=fmt, ctrl="separable", fixed_w=1, sep_q=q)
    plan = td.tdgemm_plan(desc, Ad, Bd, None)
    sa, sb, pairs, _ = td.tdgemm_plan_export(plan)
    nI, nL, nJ, npairs = plan.dims
    for i in range(nI):
        for l in range(nL):
            o = ref.stats_a[i][l]
            assert (sa[i, l]["mn"], sa[i, l]["mx"], sa[i, l]["sumsq"], sa[i, l]["n"]) == (o.mn, o.mx, o.sumsq, o.n)
    for l in range(nL):
        for j in range(nJ):
            o = ref.stats_b[l][j]
            assert (sb[l, j]["mn"], sb[l, j]["mx"], sb[l, j]["sumsq"], sb[l, j]["n"]) == (o.mn, o.mx, o.sumsq, o.n)
    for (i, j, l), o in ref.options.items():
        g = pairs[i, j, l]
        assert int(g["w"]) == 1 and int(g["p"]) == o.p
        for f in ("c_a", "c_b", "inv", "d", "r_max", "s_rep", "q_a", "q_b"):
            assert float(g[f]) == float(getattr(o, f)), (f, i, j, l)

    sh = td.block_scaled_shapes(plan)
    qA = torch.full(sh["qA"], 0xAB, dtype=torch.uint8, device="cuda")
    qB = torch.full(sh["qB"], 0xAB, dtype=torch.uint8, device="cuda")
    td.tdgemm_compand(plan, Ad, Bd, qA, qB)
    prod_dt = torch.int32 if fmt == "i8" else torch.float32
    R = torch.full(sh["products"], -7, dtype=prod_dt, device="cuda")
    td.tdgemm_gemm(plan, qA, qB, R, fused=0)
    C_st = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
    C_fu = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
    td.tdgemm_unpack(plan, R, None, C_st)
    td.tdgemm_gemm(plan, qA, qB, C_fu, fused=1)
    torch.cuda.synchronize()

    np.testing.assert_array_equal(qA.cpu().numpy(), pr.codes(ref.qa, fmt))
    np.testing.assert_array_equal(qB.cpu().numpy(), pr.codes(ref.qb, fmt).T)
    Rh = R.cpu().numpy()
    for (i, j, l), r in ref.products.items():
        p = (i * nJ + j) * nL + l
        if fmt == "i8":
            np.testing.assert_array_equal(Rh[p].astype(np.int64), r, err_msg=f"pair {p}")
        else:
            a = ref.qa[i * 128:(i + 1) * 128, l * 128:(l + 1) * 128]
            b = ref.qb[l * 128:(l + 1) * 128, j * 128:(j + 1) * 128]
            big = np.max(np.abs(a)[:, :, None] * np.abs(b)[None, :, :], axis=1)
            exact = a @ b                  # exact in float64 (products of E4M3 values)
            assert np.all(np.abs(Rh[p].astype(np.float64) - exact) <= 2.0 ** -10 * big), p
    cst, cfu = C_st.cpu().numpy(), C_fu.cpu().numpy()
    np.testing.assert_array_equal(cst, cfu)
    if fmt == "i8":
        np.testing.assert_array_equal(cfu, ref.C)
    else:
        assert rel_err(cfu, ref.C) <= 1e-4
    exact = A.astype(np.float64) @ B.astype(np.float64)
    snr = 10 * math.log10(float(np.sum(exact ** 2)) / float(np.sum((cfu - exact) ** 2)))
    log(f"[precision] {name}: SNR vs FP64 {snr:.2f} dB, rel err vs oracle {rel_err(cfu, ref.C):.2e}")


def test_block_scaled_empty_and_k0(td):
    for (M, K, N) in [(0, 50, 30), (40, 0, 30), (40, 50, 0)]:
        A = torch.ones((M, K), dtype=torch.float64, device="cuda")
        B = torch.ones((K, N), dtype=torch.float64, device="cuda")
        C, plan, qA, qB = td.block_scaled_matmul(A, B, "i8")
        torch.cuda.synchronize()
        assert C.shape == (M, N) and (C.numel() == 0 or float(C.abs().max()) == 0.0)


def test_block_scaled_rejects_bad_descriptors(td):
    A = torch.ones((130, 130), dtype=torch.float64, device="cuda")
    for kw, status in [(dict(L=64), "TDGEMM_E_UNSUPPORTED"), (dict(sep_q=200.0), "TDGEMM_E_ARG"),
                       (dict(fixed_w=2), "TDGEMM_E_ARG"), (dict(ctrl="snr"), "TDGEMM_E_ARG")]:
        args = dict(L=128, prec="i8", ctrl="separable", fixed_w=1, sep_q=127.0)
        args.update(kw)
        desc = td.make_desc(A, A, **args)
        with pytest.raises(td.TdgemmError) as e:
            td.tdgemm_plan(desc, A, A, None)
        assert status in str(e.value)


@pytest.mark.parametrize("fmt,q", [("i8", 127.0), ("e4m3", 448.0)])
def test_block_scaled_plan_query(td, fmt, q):
    """tdgemm_plan_query on the block-scaled form: every pair W = 1, and the
    predicted SNR from the oracle's records (signal L_eff sigma_a^2 sigma_b^2 over D)."""
    M, K, N = 300, 400, 260
    A, B = _inputs(M, K, N, np.float64, 17)
    ref = pr.run(A, B, 128, fmt, q, keep_products=False)
    Ad, Bd = to_dev(A), to_dev(B)
    desc = td.make_desc(Ad, Bd, L=128, prec=fmt, ctrl="separable", fixed_w=1, sep_q=q)
    plan = td.tdgemm_plan(desc, Ad, Bd, None)
    got_snr, hist, short = td.tdgemm_plan_query(plan)
    nI, nL, nJ, npairs = plan.dims
    assert hist.tolist() == [0, npairs, 0, 0, 0] and short == 0
    sig, noise = [], []
    for (i, j, l), o in ref.options.items():
        sa, sb = ref.stats_a[i][l], ref.stats_b[l][j]
        va = sa.sumsq / sa.n if sa.n else 0.0
        vb = sb.sumsq / sb.n if sb.n else 0.0
        sig.append(min(128, K - l * 128) * va * vb)
        noise.append(o.d)
    n_sum = math.fsum(noise)
    want = math.inf if n_sum == 0.0 else 10.0 * math.log10(math.fsum(sig) / n_sum)
    assert (got_snr == want) if math.isinf(want) else abs(got_snr - want) <= 1e-9
    log(f"[precision] plan query {fmt}: predicted SNR {got_snr:.2f} dB")
