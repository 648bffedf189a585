"""The pins catch plausible mistakes: each test plants one mistake in the oracle
(on the CPU, by monkeypatching a function for the duration of the test) and
checks that the corresponding pin then fails."""
import math

import numpy as np
import pytest

from oracle import blocks as bk
from oracle import control as ct
from oracle import exactsum
from oracle import noise as nz
from oracle import packing as pk
from tests import test_oracle_blocks as tb
from tests import test_oracle_control as tc
from tests import test_oracle_noise as tn
from tests import test_oracle_packing as tp


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_pack_b_with_wrong_weight_direction(monkeypatch):
    orig = pk.pack_sym_b
    monkeypatch.setattr(pk, "pack_sym_b", lambda qb, W, p, prec: orig(qb, W, -p, prec))
    _fails(tp.test_packed_words_and_eq8_expansion_exact, 2)


def test_pack_a_wrong_slot_order(monkeypatch):
    orig = pk.pack_sym_a
    monkeypatch.setattr(pk, "pack_sym_a", lambda qa, W, p, prec: orig(qa[:, ::-1].copy(), W, p, prec)[:, ::-1].copy())
    _fails(tp.test_packed_words_and_eq8_expansion_exact, 2)


def test_unpack_sym_drops_side_output_removal(monkeypatch):
    monkeypatch.setattr(pk, "unpack_sym", lambda rbar, p, prec: np.rint(rbar))
    _fails(tp.test_unpack_equals_bruteforce_in_exact_regime, "sym", "f64", 2, 64, 100)


def test_unpack_sym_wrong_sign(monkeypatch):
    def bad(rbar, p, prec):
        u = np.rint(rbar)
        return u + 2.0 ** p * np.rint(2.0 ** -p * u)
    monkeypatch.setattr(pk, "unpack_sym", bad)
    _fails(tp.test_unpack_sym_handbuilt)


def test_unpack_asym_wrong_row_order(monkeypatch):
    orig = pk.unpack_asym
    monkeypatch.setattr(pk, "unpack_asym", lambda rbar, W, p, prec: orig(rbar, W, p, prec)[::-1].copy())
    _fails(tp.test_unpack_asym_handbuilt)


def test_packing_exponent_off_by_one(monkeypatch):
    orig = pk.packing_exponent
    monkeypatch.setattr(pk, "packing_exponent", lambda r, u_safe=50.0: orig(r, u_safe) - 1)
    _fails(tp.test_prop1_numbers_by_hand)


def test_compand_floor_instead_of_round(monkeypatch):
    monkeypatch.setattr(pk, "compand", lambda X, c, prec: np.floor(pk.DTYPES[prec](c) * np.asarray(X, dtype=pk.DTYPES[prec])))
    _fails(tn.test_prop2_quantization_noise_monte_carlo, "gauss")


def test_noise_model_dropped_cross_term(monkeypatch):
    def bad(L, s_a, s_b, c_a, c_b):
        na, nb = nz.sigma_nu(c_a), nz.sigma_nu(c_b)
        return L * ((s_a * nb) ** 2 + (na * nb) ** 2)
    monkeypatch.setattr(nz, "quant_noise_eq19", bad)
    _fails(tn.test_prop2_quantization_noise_monte_carlo, "gauss")


def test_companders_swapped(monkeypatch):
    monkeypatch.setattr(nz, "companders_eq26", lambda s_a, s_b, c: (np.sqrt(s_a / (s_b * c)), np.sqrt(s_b / (s_a * c))))
    _fails(tn.test_prop4_identities)


def test_nsr_without_1_over_L(monkeypatch):
    def bad(L, s_a, s_b, c_tot, s_rep):
        ss = s_a * s_b
        return c_tot / (6 * ss) + c_tot ** 2 / (144 * ss * ss) + s_rep ** 2 * c_tot ** 2 / (ss * ss)
    monkeypatch.setattr(nz, "nsr_prop4", bad)
    _fails(tn.test_nsr_reading_equals_eq21_at_eq26_and_scale_invariance)


def test_prune_removes_smallest(monkeypatch):
    def bad(options, w_desc, d_kernel):
        nl = len(options)
        level = [0] * nl
        d = [options[l][w_desc[0]].d for l in range(nl)]
        while exactsum.exact_sum(d) > d_kernel:
            cand = [l for l in range(nl) if level[l] < len(w_desc) - 1]
            if not cand:
                break
            lstar = min(cand, key=lambda l: d[l])
            level[lstar] += 1
            d[lstar] = options[lstar][w_desc[level[lstar]]].d
        return [w_desc[level[l]] for l in range(nl)]
    monkeypatch.setattr(ct, "prune", bad)
    _fails(tc.test_prune_two_levels_closed_form)


def test_sum_of_squares_naive(monkeypatch):
    monkeypatch.setattr(tb, "sum_of_squares", lambda x: float(np.sum(np.asarray(x) ** 2)))
    _fails(tb.test_sum_of_squares_absorption_case)


def test_stats_including_padding(monkeypatch):
    def bad(X, r, c, L):
        sub = bk.block(np.asarray(X, dtype=np.float64), r, c, L)
        return bk.BlockStats(float(sub.min()), float(sub.max()), exactsum.sum_of_squares(sub), int(sub.size))
    monkeypatch.setattr(bk, "block_stats", bad)
    _fails(tb.test_block_stats_definitions)


# --- INT8 / FP8 block-scaled form
from oracle import precision as pr  # noqa: E402
from tests import test_oracle_precision as tq  # noqa: E402


def test_e4m3_ties_away_from_zero(monkeypatch):
    def away(v):
        a = abs(v)
        if a == 0.0 or a >= 448.0:
            return orig(v)
        e = np.frexp(a)[1] - 1
        step = 2.0 ** -9 if a < 2.0 ** -6 else 2.0 ** (e - 3)
        return float(np.copysign(min(np.floor(a / step + 0.5) * step, 448.0), v))
    orig = pr.e4m3_round
    monkeypatch.setattr(pr, "e4m3_round", away)
    _fails(tq.test_e4m3_round_nearest_even_brute_force)


def test_e4m3_wrong_bias(monkeypatch):
    orig = pr.e4m3_decode
    monkeypatch.setattr(pr, "e4m3_decode", lambda c: orig(c) * 2.0)
    _fails(tq.test_e4m3_code_table)


def test_block_scale_from_rms_instead_of_range(monkeypatch):
    monkeypatch.setattr(pr, "block_scale", lambda st, q: 0.0 if st.amax == 0 else q / (3.0 * st.sigma))
    _fails(tq.test_integer_blocks_at_full_range_are_exact)


def test_int8_truncation_instead_of_rounding(monkeypatch):
    orig = pr.quantize_block
    monkeypatch.setattr(pr, "quantize_block",
                        lambda x, c, fmt: np.trunc(np.asarray(x) * c) if fmt == "i8" else orig(x, c, fmt))
    _fails(tq.test_int8_snr_matches_prop2, "laplace")


def test_prune_accel_removes_smallest(monkeypatch):
    def wrong(options, w_desc, frac):
        nl = len(options)
        order = sorted(range(nl), key=lambda l: (options[l][w_desc[0]].d, l))   # smallest first
        need = math.ceil(frac * nl - 1e-12)
        keep = set(order[len(order) - need:]) if need else set()
        return [w_desc[0] if l in keep else w_desc[-1] for l in range(nl)]
    monkeypatch.setattr(ct, "prune_accel", wrong)
    _fails(tc.test_prune_accel_two_levels_is_the_cheapest_fraction)
