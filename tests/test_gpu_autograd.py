"""The autograd linear layer through the C-ABI: finite differences on the
unquantized path, packed gradients against the oracle and the FP64 reference
(distortion stated), and a few training steps of a perceptron."""
import math

import numpy as np
import pytest

from oracle import pipeline as pl
from tests.gpu_common import assert_elementwise, device_calib, log, oracle_cfg, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ag():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1110_5765_amd import autograd, tdgemm
    return autograd, tdgemm


def test_gradcheck_unquantized(ag):
    """W = 1 everywhere is the native product: torch.autograd.gradcheck (central
    finite differences in FP64) must agree with the packed backward."""
    autograd, _ = ag
    tdc = autograd.TDContext(autograd.TDConfig(prec="f64", ctrl="fixed", fixed_w=1, min_dim=1), None)
    g = torch.Generator(device="cpu").manual_seed(3)
    X = torch.randn(24, 20, dtype=torch.float64, generator=g).cuda().requires_grad_()
    W = torch.randn(20, 18, dtype=torch.float64, generator=g).cuda().requires_grad_()
    b = torch.randn(18, dtype=torch.float64, generator=g).cuda().requires_grad_()
    assert torch.autograd.gradcheck(lambda x, w, bb: autograd.TDLinearFn.apply(x, w, bb, tdc),
                                    (X, W, b), eps=1e-6, atol=1e-8, rtol=1e-6)
    assert tdc.calls > 0 and tdc.plain_calls == 0


@pytest.mark.parametrize("snr", [25.0, 40.0])
def test_packed_gradients_vs_oracle_and_fp64(ag, snr):
    """FP32 packing (sym, L = 64, W in {1, 2}) at S dB per inner kernel. The
    three products equal the oracle's (1e-5 relative); their SNR against FP64
    is logged and must be within 3 dB of the target (the per-inner-kernel
    budget is met in expectation)."""
    autograd, td = ag
    L = 64
    calib, tabs = device_calib(td, L, "sym", "f32", (2,))
    cfg = autograd.TDConfig(L=L, form="sym", prec="f32", ctrl="snr", snr_db=snr, w_allowed=(1, 2),
                            min_dim=64)
    tdc = autograd.TDContext(cfg, calib)
    rng = np.random.default_rng(int(snr))
    X = rng.standard_normal((256, 192)).astype(np.float32)
    W = (rng.standard_normal((192, 320)) / math.sqrt(192)).astype(np.float32)
    G = rng.standard_normal((256, 320)).astype(np.float32)
    Xd = torch.from_numpy(X).cuda().requires_grad_()
    Wd = torch.from_numpy(W).cuda().requires_grad_()
    Y = autograd.TDLinearFn.apply(Xd, Wd, None, tdc)
    Y.backward(torch.from_numpy(G).cuda())
    torch.cuda.synchronize()
    ocfg = oracle_cfg(L, "sym", "f32", "snr", snr, (1, 2), 2, 1.0, 127.0)
    got = {"Y": Y.detach().cpu().numpy(), "dX": Xd.grad.cpu().numpy(), "dW": Wd.grad.cpu().numpy()}
    import dataclasses

    def oracle(a, b):      # the library groups the l-sum as auto_k_split says
        ks = td.auto_k_split(a.shape[0], b.shape[1], a.shape[1], L, "f32")
        return pl.run(a, b, dataclasses.replace(ocfg, k_groups=ks), calib=tabs).C

    operands = {"Y": (X, W), "dX": (G, W.T.copy()), "dW": (X.T.copy(), G)}
    ref = {k: oracle(a, b) for k, (a, b) in operands.items()}
    exact = {"Y": X.astype(np.float64) @ W, "dX": G.astype(np.float64) @ W.T.astype(np.float64),
             "dW": X.T.astype(np.float64) @ G}
    for k in ("Y", "dX", "dW"):
        # bit for bit with the oracle's grouping of the l-sum, and element by element
        # within 1e-5 |A||B| of eq. (2) as one ascending sum
        np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
        a, b = operands[k]
        assert_elementwise(got[k], pl.run(a, b, ocfg, calib=tabs).C, a, b, 1e-5, f"{k} vs the ascending l-sum")
        assert rel_err(got[k], ref[k]) <= 1e-5, k
        s = pl.snr_db(got[k].astype(np.float64), exact[k])
        log(f"[autograd] S={snr:g}: {k} SNR vs FP64 {s:.2f} dB")
        assert s >= snr - 3.0, (k, s)


def test_int8_block_scaled_layer_vs_oracle(ag):
    """prec "i8": the layer's three products in the INT8 block-scaled form
    (Remark 1) equal the oracle's block-scaled product bit for bit (ragged
    shapes, transposed operands as views); their SNR against FP64 is logged."""
    from oracle import precision as pr
    autograd, td = ag
    cfg = autograd.TDConfig(L=128, prec="i8", ctrl="separable", sep_q=127.0, min_dim=64)
    tdc = autograd.TDContext(cfg, None)
    rng = np.random.default_rng(8)
    X = rng.standard_normal((300, 200)).astype(np.float32)
    W = (rng.standard_normal((200, 260)) / math.sqrt(200)).astype(np.float32)
    G = rng.laplace(0.0, 1.0, (300, 260)).astype(np.float32)
    Xd = torch.from_numpy(X).cuda().requires_grad_()
    Wd = torch.from_numpy(W).cuda().requires_grad_()
    Y = autograd.TDLinearFn.apply(Xd, Wd, None, tdc)
    Y.backward(torch.from_numpy(G).cuda())
    torch.cuda.synchronize()
    assert tdc.calls == 3 and tdc.plain_calls == 0
    got = {"Y": Y.detach().cpu().numpy(), "dX": Xd.grad.cpu().numpy(), "dW": Wd.grad.cpu().numpy()}
    operands = {"Y": (X, W), "dX": (G, W.T.copy()), "dW": (X.T.copy(), G)}
    for k, (a, b) in operands.items():
        ref = pr.run(a.astype(np.float64), b.astype(np.float64), 128, "i8", 127.0).C
        np.testing.assert_array_equal(got[k], ref, err_msg=k)
        exact = a.astype(np.float64) @ b.astype(np.float64)
        log(f"[autograd] INT8 block-scaled {k}: SNR vs FP64 {pl.snr_db(got[k].astype(np.float64), exact):.2f} dB")


def test_mlp_steps_track_plain(ag):
    """A 512 -> 256 -> 10 perceptron, 20 SGD steps from the same start: the
    packed model's loss follows the plain FP32 model's closely and decreases."""
    autograd, td = ag
    L = 64
    calib, _ = device_calib(td, L, "sym", "f32", (2,))
    tdc = autograd.TDContext(autograd.TDConfig(L=L, prec="f32", snr_db=30.0, w_allowed=(1, 2)), calib)
    g = torch.Generator(device="cpu").manual_seed(5)
    W1 = (torch.rand(512, 256, generator=g) * 2 - 1) * math.sqrt(6 / 768)
    W2 = (torch.rand(256, 10, generator=g) * 2 - 1) * math.sqrt(6 / 266)
    X = torch.randn(1024, 512, generator=g).cuda()
    y = torch.randint(0, 10, (1024,), generator=g).cuda()

    def train(packed):
        w1 = W1.clone().cuda().requires_grad_()
        w2 = W2.clone().cuda().requires_grad_()
        losses = []
        for _ in range(20):
            h = autograd.TDLinearFn.apply(X, w1, None, tdc) if packed else X @ w1
            h = torch.relu(h)
            out = autograd.TDLinearFn.apply(h, w2, None, tdc) if packed else h @ w2
            loss = torch.nn.functional.cross_entropy(out, y)
            w1.grad = w2.grad = None
            loss.backward()
            with torch.no_grad():
                w1 -= 0.5 * w1.grad
                w2 -= 0.5 * w2.grad
            losses.append(float(loss))
        return losses

    lp, lq = train(False), train(True)
    log(f"[autograd] MLP loss plain {lp[0]:.4f} -> {lp[-1]:.4f}, packed {lq[0]:.4f} -> {lq[-1]:.4f}")
    assert lq[-1] < lq[0] - 0.05
    assert max(abs(a - b) for a, b in zip(lp, lq)) < 0.02
    assert tdc.calls > 0
