"""Pins of the oracle's noise model and companders (Props. 2-4, eqs. 19-27).

* Prop. 2 / eq. (19) against Monte Carlo: i.i.d. Gaussian and Laplacian
  blocks run through the oracle's compand -> pack -> product -> unpack ->
  de-compand path (exact regime, no representation error); the measured MSE
  against the exact FP64 product must match the closed form within 3 %.
* Prop. 4 / eq. (26): the companders' product and ratio identities, the
  minimum of the eq. (21) noise over the compander ratio (a numerical sweep),
  and the double root of eq. (34) at which Prop. 3 collapses onto Prop. 4.
* The eq. (27) noise as read here equals eq. (21) evaluated at eq. (26), is
  invariant to A -> tA, and matches measured SNR within 0.5 dB (Fig. 4 protocol
  with s = 0).
* Independence of quantization and representation error (Sec. 5.A): Pearson
  correlation below 1e-2.
"""
import math

import numpy as np
import pytest

from oracle import noise as nz
from oracle import packing as pk
from oracle.blocks import block_stats


def _draw(dist, rng, shape):
    return rng.standard_normal(shape) if dist == "gauss" else rng.laplace(0.0, 1.0, shape)


def _pair_sym(a, b, c_a, c_b, W, prec="f64"):
    qa = pk.compand(a, c_a, prec)
    qb = pk.compand(b, c_b, prec)
    L = a.shape[0]
    qmax = max(np.abs(qa).max(), np.abs(qb).max())
    p = pk.packing_exponent(float(L) * float(np.abs(qa).max()) * float(np.abs(qb).max()))
    rbar = pk.packed_product(pk.pack_sym_a(qa, W, p, prec), pk.pack_sym_b(qb, W, p, prec), prec)
    r = pk.unpack_sym(rbar, p, prec)
    return pk.decompand(r, 1.0 / (c_a * c_b), prec), qa, qb, qmax, p


@pytest.mark.parametrize("dist", ["gauss", "laplace"])
def test_prop2_quantization_noise_monte_carlo(dist):
    rng = np.random.default_rng(2024 if dist == "gauss" else 2025)
    L, W, npairs = 64, 2, 120
    sq = []
    sigma = 1.0 if dist == "gauss" else math.sqrt(2.0)
    c = 25.0 / sigma                     # c * sigma >> 1: the uniform-noise model holds
    for _ in range(npairs):
        a = _draw(dist, rng, (L, L))
        b = _draw(dist, rng, (L, L))
        rhat, qa, qb, qmax, p = _pair_sym(a, b, c, c, W)
        assert pk.exact_regime_sym(L // W, np.abs(qa).max(), np.abs(qb).max(), W, p,
                                   L * np.abs(qa).max() * np.abs(qb).max(), "f64")
        np.testing.assert_array_equal(pk.unpack_sym(
            pk.packed_product(pk.pack_sym_a(qa, W, p, "f64"), pk.pack_sym_b(qb, W, p, "f64"), "f64"),
            p, "f64").astype(np.int64), qa.astype(np.int64) @ qb.astype(np.int64))
        sq.append(((rhat - a @ b) ** 2).ravel())
    mse = float(np.mean(np.concatenate(sq)))
    # eq. (19) written out: L [(s_a s_nb)^2 + (s_b s_na)^2 + (s_na s_nb)^2], s_n = 1/(c sqrt 12)
    sn = 1.0 / (c * math.sqrt(12.0))
    want = L * (2 * (sigma * sn) ** 2 + sn ** 4)
    assert abs(mse / want - 1.0) < 0.03
    assert abs(nz.quant_noise_eq19(L, sigma, sigma, c, c) / want - 1.0) < 1e-12


def test_prop4_identities():
    s_a, s_b, ctot = 0.7, 2.3, 1e-3
    c_a, c_b = nz.companders_eq26(s_a, s_b, ctot)
    assert abs(c_a * c_b * ctot - 1.0) < 1e-14          # c_A c_B = 1 / c_tot (eqs. 17, 24)
    assert abs((c_a / c_b) / (s_b / s_a) - 1.0) < 1e-14  # c_A / c_B = s_b / s_a


def test_prop4_is_minimum_of_eq21():
    """Sweep the ratio c_A / c_B at fixed c_A c_B = 1/c_tot; eq. (21) is smallest at eq. (26)."""
    L, s_a, s_b, ctot, s_rep = 64.0, 0.5, 3.0, 2e-4, 0.0
    ratios = np.exp(np.linspace(-4, 4, 4001))
    noise = []
    for rr in ratios:
        c_a = math.sqrt(rr / ctot)
        c_b = 1.0 / (ctot * c_a)
        sna, snb = 1 / (c_a * math.sqrt(12)), 1 / (c_b * math.sqrt(12))
        noise.append(L * ((s_a * snb) ** 2 + (s_b * sna) ** 2 + (sna * snb) ** 2) + (s_rep / (c_a * c_b)) ** 2)
    best = ratios[int(np.argmin(noise))]
    assert abs(best / (s_b / s_a) - 1.0) < 5e-3


def test_prop3_double_root_is_prop4():
    """Eq. (25) with equality: the two compander solutions of eq. (22) coincide with eq. (26)."""
    L, s_a, s_b, ctot, s_rep = 64.0, 1.3, 0.4, 5e-4, 0.7
    # the SNR at which D_QvR = 2 s_a s_b c_tot (the maximum of eq. 27)
    nsr = nz.nsr_prop4(L, s_a, s_b, ctot, s_rep)
    snr = -10.0 * math.log10(nsr)
    d = nz.d_qvr_eq23(L, s_a, s_b, snr, ctot, s_rep)
    assert abs(d / (2 * s_a * s_b * ctot) - 1.0) < 1e-9
    c4 = nz.companders_eq26(s_a, s_b, ctot)
    # a hair below the maximum the two roots straddle eq. (26)
    lo = nz.companders_eq22(L, s_a, s_b, snr - 1e-6, ctot, s_rep, -1)
    hi = nz.companders_eq22(L, s_a, s_b, snr - 1e-6, ctot, s_rep, +1)
    assert lo is not None and hi is not None
    assert lo[0] < c4[0] < hi[0]
    assert abs(lo[0] / c4[0] - 1) < 1e-2 and abs(hi[0] / c4[0] - 1) < 1e-2
    # above the maximum no admissible companders exist (eq. 25)
    assert nz.companders_eq22(L, s_a, s_b, snr + 0.5, ctot, s_rep) is None
    # any admissible pair reaches the requested SNR through eq. (21)
    c_a, c_b = nz.companders_eq22(L, s_a, s_b, snr - 3.0, ctot, s_rep, +1)
    assert abs(c_a * c_b * ctot - 1) < 1e-12
    got = nz.snr_eq20(L, s_a, s_b, nz.combined_noise_eq21(L, s_a, s_b, c_a, c_b, s_rep))
    assert abs(got - (snr - 3.0)) < 1e-9


def test_nsr_reading_equals_eq21_at_eq26_and_scale_invariance():
    L, s_a, s_b, amax_a, amax_b, R, s_rep = 64.0, 0.9, 1.7, 4.1, 6.2, 3e6, 2.5
    ctot = nz.c_tot_eq24(L, amax_a, amax_b, R)
    c_a, c_b = nz.companders_eq26(s_a, s_b, ctot)
    d = nz.combined_noise_eq21(L, s_a, s_b, c_a, c_b, s_rep)
    signal = L * (s_a * s_b) ** 2
    assert abs(nz.nsr_prop4(L, s_a, s_b, ctot, s_rep) / (d / signal) - 1) < 1e-12
    for t in (1e-3, 7.0, 1e5):
        ct2 = nz.c_tot_eq24(L, t * amax_a, amax_b, R)
        assert abs(nz.nsr_prop4(L, t * s_a, s_b, ct2, s_rep) / nz.nsr_prop4(L, s_a, s_b, ctot, s_rep) - 1) < 1e-12


@pytest.mark.parametrize("R", [2.0 ** 14, 2.0 ** 17, 2.0 ** 20])
def test_eq27_matches_measured_snr(R):
    """Fig. 4 protocol with s = 0: companders from eq. (26) per R, measured SNR vs model."""
    rng = np.random.default_rng(int(R))
    L, W = 64, 2
    sig, err, nsr_terms = 0.0, 0.0, []
    for _ in range(60):
        a = rng.standard_normal((L, L))
        b = rng.standard_normal((L, L))
        sa, sb = block_stats(a, 0, 0, L), block_stats(b, 0, 0, L)
        ctot = nz.c_tot_eq24(L, sa.amax, sb.amax, R)
        c_a, c_b = nz.companders_eq26(sa.sigma, sb.sigma, ctot)
        rhat = _pair_sym(a, b, c_a, c_b, W)[0]
        ref = a @ b
        sig += float(np.sum(ref ** 2))
        err += float(np.sum((rhat - ref) ** 2))
        nsr_terms.append(nz.nsr_prop4(L, sa.sigma, sb.sigma, ctot, 0.0))
    measured = 10 * math.log10(sig / err)
    model = -10 * math.log10(float(np.mean(nsr_terms)))
    assert abs(measured - model) < 0.5


def test_quantization_and_representation_errors_uncorrelated():
    """Sec. 5.A: Pearson |corr(eps_quant, eps_repr)| < 1e-2 (FP32, W = 2, beyond the exact regime)."""
    rng = np.random.default_rng(77)
    L, W = 64, 2
    eq, er = [], []
    for _ in range(80):
        a = rng.standard_normal((L, L))
        b = rng.standard_normal((L, L))
        c = 12.0
        qa = pk.compand(a, c, "f32")
        qb = pk.compand(b, c, "f32")
        p = pk.packing_exponent(float(L) * np.abs(qa).max() * np.abs(qb).max())
        r = pk.unpack_sym(pk.packed_product(pk.pack_sym_a(qa, W, p, "f32"), pk.pack_sym_b(qb, W, p, "f32"), "f32"), p, "f32")
        exact = (qa.astype(np.int64) @ qb.astype(np.int64)).astype(np.float64)
        eq.append((exact / c ** 2 - a @ b).ravel())
        er.append(((r.astype(np.float64) - exact) / c ** 2).ravel())
    eq, er = np.concatenate(eq), np.concatenate(er)
    assert np.std(er) > 0, "representation errors must be present for the test to mean anything"
    corr = float(np.corrcoef(eq, er)[0, 1])
    assert abs(corr) < 1e-2
