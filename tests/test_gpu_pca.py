"""GPU parity of the 2D-PCA application's GEMMs (Sec. 8.A) on synthetic images.

The image scatter matrix G = sum_j A_j^T A_j (one product over the stacked
training images, A^T passed as a transposed view) and the projections Y = A X
run through the library with FP32 packing at L = 96 and are compared with the
oracle on the same inputs; X comes from the oracle's G, so both sides project
onto the same axes. G sums its 12 subblocks in groups (auto_k_split), as the
bench does. Bar: relative Frobenius error <= 1e-5 (FP32 packing), and
the nearest-neighbour matches of the two sides agree.
"""
import numpy as np
import pytest

import workloads
from oracle import pipeline as pl
from tests.gpu_common import assert_elementwise, device_calib, log, oracle_cfg, rel_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def td():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1110_5765_amd import tdgemm
    return tdgemm


@pytest.mark.parametrize("snr", [25.0, 15.0])
def test_pca2d_gemms(td, snr):
    L, d, size = 96, 6, 96
    tr, ltr, te, lte = workloads.faces(n_person=4, n_train=3, n_test=2, size=size)
    mu = tr.mean(0)
    S = (tr - mu).reshape(-1, size).astype(np.float32)          # 1152 x 96
    T = (te - mu).reshape(-1, size).astype(np.float32)          # 768 x 96
    log(f"[pca] S {S.shape} T {T.shape} snr={snr}")
    calib, tabs = device_calib(td, L, "sym", "f32", (2,))
    cfg = oracle_cfg(L, "sym", "f32", "snr", snr, (1, 2), 2, 1.0, 127.0)

    def ks(A, B):
        return td.auto_k_split(A.shape[0], B.shape[1], A.shape[1], L, "f32")

    def lib(A, B):
        desc = td.make_desc(A, B, L=L, form="sym", prec="f32", ctrl="snr", snr_db=snr, w_allowed=(1, 2),
                            k_split=ks(A, B))
        plan = td.tdgemm_plan(desc, A, B, calib)
        C = torch.empty((A.shape[0], B.shape[1]), dtype=torch.float32, device="cuda")
        td.tdgemm_gemm(plan, A, B, C, fused=1)
        torch.cuda.synchronize()
        return C.cpu().numpy()

    Sd, Td = to_dev(S), to_dev(T)
    import dataclasses
    G_ref = pl.run(np.ascontiguousarray(S.T), S, dataclasses.replace(cfg, k_groups=ks(Sd.t(), Sd)),
                   calib=tabs).C
    G = lib(Sd.t(), Sd)
    # bit for bit with the oracle's grouping of the l-sum, element by element within
    # 1e-5 |A||B| of eq. (2) as one ascending sum
    St = np.ascontiguousarray(S.T)
    np.testing.assert_array_equal(G, G_ref)
    assert_elementwise(G, pl.run(St, S, cfg, calib=tabs).C, St, S, 1e-5, "G vs the ascending l-sum")
    assert rel_err(G, G_ref) <= 1e-5
    _, V = np.linalg.eigh(G_ref.astype(np.float64))
    X = np.ascontiguousarray(V[:, ::-1][:, :d]).astype(np.float32)
    Xd = to_dev(X)
    Ys_ref = pl.run(S, X, dataclasses.replace(cfg, k_groups=ks(Sd, Xd)), calib=tabs).C
    Yt_ref = pl.run(T, X, dataclasses.replace(cfg, k_groups=ks(Td, Xd)), calib=tabs).C
    Ys, Yt = lib(Sd, Xd), lib(Td, Xd)
    np.testing.assert_array_equal(Ys, Ys_ref)
    np.testing.assert_array_equal(Yt, Yt_ref)
    assert_elementwise(Ys, pl.run(S, X, cfg, calib=tabs).C, S, X, 1e-5, "Ys vs the ascending l-sum")
    assert_elementwise(Yt, pl.run(T, X, cfg, calib=tabs).C, T, X, 1e-5, "Yt vs the ascending l-sum")
    assert rel_err(Ys, Ys_ref) <= 1e-5 and rel_err(Yt, Yt_ref) <= 1e-5

    def match(ys, yt):
        a = yt.reshape(te.shape[0], -1).astype(np.float64)
        b = ys.reshape(tr.shape[0], -1).astype(np.float64)
        return (((a[:, None, :] - b[None, :, :]) ** 2).sum(-1)).argmin(1)

    m_lib, m_ref = match(Ys, Yt), match(Ys_ref, Yt_ref)
    assert np.array_equal(m_lib, m_ref)
    G64 = S.T.astype(np.float64) @ S.astype(np.float64)
    log(f"[pca] snr={snr}: SNR(G) {pl.snr_db(G, G64):.2f} dB, recognition "
        f"{100 * float((ltr[m_lib] == lte).mean()):.1f} %")
