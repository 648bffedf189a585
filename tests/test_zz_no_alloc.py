"""The allocation-free entry point tdgemm_matmul_noalloc, called through the
C-ABI, against tdgemm_plan + tdgemm_gemm(fused = 1) with a caller workspace:
the same kernels on the same inputs, so C must match bit for bit. Two calls in
a row share the library's static workspace; the second is smaller and uses a
split l-sum (its partial results live in that workspace too)."""
import numpy as np
import pytest

from tests.gpu_common import device_calib, log, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def td():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1110_5765_amd import tdgemm
    return tdgemm


CALLS = [
    # name, M, K, N, L, form, prec (inputs and packing), S, W allowed, k_split
    ("big_L64_sym", 700, 900, 650, 64, "sym", "f64", 40.0, (1, 2, 4), 1),
    ("small_L128_asym_split", 200, 128 * 7 + 30, 150, 128, "asym", "f64", 30.0, (1, 2, 4), 3),
    ("f32_L96", 190, 300, 210, 96, "sym", "f32", 15.0, (1, 2), 1),
]


def _run_pair(td, case):
    name, M, K, N, L, form, prec, snr, wal, ks = case
    log(f"[noalloc] {name}: M={M} K={K} N={N} L={L} {form} {prec} S={snr} k_split={ks}")
    dt = np.float64 if prec == "f64" else np.float32
    r = np.random.default_rng(M + K + N)
    A = to_dev(r.standard_normal((M, K)).astype(dt))
    B = to_dev(r.laplace(0.0, 1.0, (K, N)).astype(dt))
    calib, _ = device_calib(td, L, form, prec, tuple(w for w in wal if w > 1))
    desc = td.make_desc(A, B, L=L, form=form, prec=prec, ctrl="snr", snr_db=snr, w_allowed=wal,
                        k_split=ks)
    assert td.tdgemm_workspace_size(desc) <= td.NOALLOC_MAX_BYTES
    pt = torch.float64 if prec == "f64" else torch.float32
    C_ref = torch.full((M, N), float("nan"), dtype=pt, device="cuda")
    plan = td.tdgemm_plan(desc, A, B, calib)
    td.tdgemm_gemm(plan, A, B, C_ref, fused=1)
    C_na = torch.full((M, N), float("nan"), dtype=pt, device="cuda")
    td.tdgemm_matmul_noalloc(desc, A, B, calib, C_na)
    torch.cuda.synchronize()
    a, b = C_ref.cpu().numpy(), C_na.cpu().numpy()
    assert np.all(np.isfinite(a))
    assert a.tobytes() == b.tobytes(), name
    return b


def test_noalloc_matches_plan_and_gemm(td):
    for case in CALLS:
        _run_pair(td, case)


def test_noalloc_rejects_oversized_workspace(td):
    """A descriptor whose workspace exceeds the static array: TDGEMM_E_WORKSPACE."""
    A = torch.empty((4096, 4096), dtype=torch.float64, device="cuda")
    B = torch.empty((4096, 4096), dtype=torch.float64, device="cuda")
    calib, _ = device_calib(td, 64, "sym", "f64")
    desc = td.make_desc(A, B, L=64, k_split=64)
    assert td.tdgemm_workspace_size(desc) > td.NOALLOC_MAX_BYTES
    C = torch.empty((4096, 4096), dtype=torch.float64, device="cuda")
    with pytest.raises(td.TdgemmError) as e:
        td.tdgemm_matmul_noalloc(desc, A, B, calib, C)
    assert e.value.status == -3
