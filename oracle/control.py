"""Per-pair option records and inner-kernel pruning (oracle; test infrastructure only).

Sec. 5.B: for every subblock pair (A_il, B_lj) and every packing W > 1 the
method computes the eq. (26) companders and {R_max*, E{S*}} (the maximum of
eq. 27), keeps them in a data structure, and prunes out the best combination
at run time. Sec. 6: per inner kernel R_ij, starting from the maximum packing,
it repeatedly removes the outcome with the highest distortion until the
inner-kernel MSE budget D_kernel(i,j) = 10^(-S/10) L sum_l (s_a,il s_b,lj)^2 is met.

Readings taken:

* R_max* is the exact argmin of the eq. (27) noise (read as in ``noise``) over
  the R values of a calibrated s(R, W) table (Sec. 4.B); ties go to the
  smaller R. The paper's nearest-neighbour lookup in an offline table keyed by
  {s_a, s_b} only approximates this argmin; under the eq. (27) reading the
  noise depends on the pair only through the range-to-RMS ratios, so the
  exact argmin costs little.
* z is computed from R_safe = L_eff Q_A Q_B with Q = [[c max|X|]], the true
  bound on the unpacked integers; eq. (17) ignores the rounding excess.
* D_W of a pair is eq. (21) at the chosen companders; W = 1 is native
  floating-point computation with D = 0. A block whose range is 0 makes the
  pair contribute nothing: c = 0, inverse 0, D = 0, at the maximum W.
* Pruning: "removing the outcome with the highest distortion" lowers that
  pair to the next smaller allowed W (ties: lowest l). Both sums of Sec. 6 are
  exactly rounded. An option a table cannot supply (no finite s(R, W), or no
  grid point where the eq. 27 noise is finite) has D = 1e300: it is removed
  first, and it is always removed, whatever the budget or the throughput
  target, because its subblock product could not be formed.
* Border pairs use L_eff, the valid inner extent, wherever L appears.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .blocks import BlockStats
from .exactsum import exact_sum
from .noise import c_tot_eq24, combined_noise_eq21, companders_eq22, companders_eq26, nsr_prop4
from .packing import packing_exponent

D_UNAVAILABLE = 1e300


@dataclass(frozen=True)
class PairOption:
    """One entry of the Sec. 5.B data structure: a pair's settings at packing W."""
    W: int
    r_max: float       # R_max* (0 for W = 1 or a zero block)
    c_a: float
    c_b: float
    q_a: float         # [[c_A max|A|]]
    q_b: float
    r_safe: float      # L_eff Q_A Q_B
    p: int             # z = 2^-p
    inv: float         # 1 / (c_A c_B)
    d: float           # expected noise power, eq. (21)
    nsr: float         # normalised noise at R_max*
    s_rep: float       # s(R_max*, W)


@dataclass(frozen=True)
class CalibTable:
    """s(R, W) of Sec. 4.B for one (form, precision, L): ascending R values with
    the measured RMSE in index units; inf marks an unusable point."""
    r: np.ndarray
    s: np.ndarray


def option_native() -> PairOption:
    """W = 1: native floating-point product, no companding."""
    return PairOption(1, 0.0, 1.0, 1.0, 0.0, 0.0, 0.0, 0, 1.0, 0.0, 0.0, 0.0)


def option_zero(W: int, u_safe: float) -> PairOption:
    """A pair with an all-zero block contributes nothing."""
    return PairOption(W, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, packing_exponent(0.0, u_safe),
                      0.0, 0.0, 0.0, 0.0)


def option_at(W: int, L_eff: int, sa: BlockStats, sb: BlockStats, r_max: float,
              s_rep: float, u_safe: float) -> PairOption:
    """Settings of one pair at packing W and range R_max (eqs. 24, 26, 15, 21)."""
    s_a, s_b = sa.sigma, sb.sigma
    ctot = c_tot_eq24(float(L_eff), sa.amax, sb.amax, r_max)
    c_a, c_b = companders_eq26(s_a, s_b, ctot)
    q_a = float(np.rint(c_a * sa.amax))
    q_b = float(np.rint(c_b * sb.amax))
    r_safe = (float(L_eff) * q_a) * q_b
    p = packing_exponent(r_safe, u_safe)
    d = combined_noise_eq21(float(L_eff), s_a, s_b, c_a, c_b, s_rep)
    nsr = nsr_prop4(float(L_eff), s_a, s_b, ctot, s_rep)
    return PairOption(W, r_max, c_a, c_b, q_a, q_b, r_safe, p, 1.0 / (c_a * c_b), d, nsr, s_rep)


def best_option(W: int, L_eff: int, sa: BlockStats, sb: BlockStats, table: CalibTable,
                u_safe: float) -> PairOption:
    """Prop. 4: the eq. (26) companders at R_max* = argmin of the eq. (27) noise."""
    if sa.amax == 0.0 or sb.amax == 0.0:
        return option_zero(W, u_safe)
    ok = np.isfinite(table.s)
    if not ok.any():
        o = option_zero(W, u_safe)
        return PairOption(W, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, o.p, 0.0, D_UNAVAILABLE, np.inf, np.inf)
    r = table.r[ok]
    s = table.s[ok]
    s_a, s_b = sa.sigma, sb.sigma
    unavailable = PairOption(W, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, option_zero(W, u_safe).p, 0.0,
                             D_UNAVAILABLE, np.inf, np.inf)
    # eq. (27) noise at every grid R, elementwise in the same operation order as nsr_prop4
    with np.errstate(over="ignore", invalid="ignore"):
        ctot = ((float(L_eff) * sa.amax) * sb.amax) / r
        ss = s_a * s_b
        t1 = ctot / (6.0 * ss)
        t2 = (ctot * ctot) / (144.0 * (ss * ss))
        t3 = ((s * s) * (ctot * ctot)) / (float(L_eff) * (ss * ss))
        nsr = (t1 + t2) + t3
    fin = np.isfinite(nsr)            # an overflowed (inf or nan) noise is no candidate
    if not fin.any():
        return unavailable
    k = int(np.flatnonzero(fin)[np.argmin(nsr[fin])])   # first minimum: the smaller R on ties
    return option_at(W, L_eff, sa, sb, float(r[k]), float(s[k]), u_safe)


def fixed_option(W: int, L_eff: int, sa: BlockStats, sb: BlockStats, r_max: float,
                 u_safe: float) -> PairOption:
    """A fixed (W, R_max) setting: eq. (26) companders, no representation term."""
    if W == 1:
        return option_native()
    if sa.amax == 0.0 or sb.amax == 0.0:
        return option_zero(W, u_safe)
    return option_at(W, L_eff, sa, sb, r_max, 0.0, u_safe)


def table_s_at(table: CalibTable, r_max: float, W: int) -> float:
    """s(R_max, W) read from a calibrated grid: the value at the smallest grid R
    not below R_max (s grows with R, so this errs on the safe side); +inf beyond
    the grid or at an unusable point."""
    k = int(np.searchsorted(table.r, r_max, side="left"))
    return float(table.s[k]) if k < table.r.size else math.inf


def target_option(W: int, L_eff: int, sa: BlockStats, sb: BlockStats, r_max: float,
                  s_rep: float, snr_db: float, u_safe: float) -> PairOption:
    """Prop. 3: a fixed (W, R_max) with the eq. (22) companders that reach the
    expected subblock SNR snr_db (the root with c_A >= c_A*, eq. 22 with +).
    When eq. (25) does not hold -- the target is beyond what R_max allows --
    the double root is taken, which is the eq. (26) pair: the highest expected
    SNR at this R_max."""
    if W == 1:
        return option_native()
    if sa.amax == 0.0 or sb.amax == 0.0:
        return option_zero(W, u_safe)
    s_a, s_b = sa.sigma, sb.sigma
    ctot = c_tot_eq24(float(L_eff), sa.amax, sb.amax, r_max)
    cc = companders_eq22(float(L_eff), s_a, s_b, snr_db, ctot, s_rep, +1)
    c_a, c_b = cc if cc is not None else companders_eq26(s_a, s_b, ctot)
    q_a = float(np.rint(c_a * sa.amax))
    q_b = float(np.rint(c_b * sb.amax))
    r_safe = (float(L_eff) * q_a) * q_b
    p = packing_exponent(r_safe, u_safe)
    d = combined_noise_eq21(float(L_eff), s_a, s_b, c_a, c_b, s_rep)
    return PairOption(W, r_max, c_a, c_b, q_a, q_b, r_safe, p, 1.0 / (c_a * c_b), d, np.nan, s_rep)


def separable_option(W: int, L_eff: int, sa: BlockStats, sb: BlockStats, q: float,
                     u_safe: float) -> PairOption:
    """Per-block companders c = Q / max|X| (Sec. 3.A uniform companding with a fixed
    integer range Q): the same integers serve every pair a block is part of."""
    if W == 1:
        return option_native()
    if sa.amax == 0.0 or sb.amax == 0.0:
        return option_zero(W, u_safe)
    c_a = q / sa.amax
    c_b = q / sb.amax
    q_a = float(np.rint(c_a * sa.amax))
    q_b = float(np.rint(c_b * sb.amax))
    r_safe = (float(L_eff) * q_a) * q_b
    p = packing_exponent(r_safe, u_safe)
    d = combined_noise_eq21(float(L_eff), sa.sigma, sb.sigma, c_a, c_b, 0.0)
    return PairOption(W, r_safe, c_a, c_b, q_a, q_b, r_safe, p, 1.0 / (c_a * c_b), d, np.nan, 0.0)


def saved_units(W: int, units: dict | None = None) -> int:
    """Work a pair saves at packing W against the W = 1 product, in integer units.

    Nominal (units None): the MFMA work, in twelfths of the W = 1 product,
    12 (1 - 1/W), an integer for every W in {1, 2, 3, 4}. Measured: Sec. 5.B
    keeps the acceleration F_W of every packing, found by off-line timing on the
    target; a pair then saves 1 - 1/F_W of its W = 1 time, which the caller
    passes quantised to integers, units[W] (W = 1 saves 0)."""
    if units is not None:
        return 0 if W == 1 else int(units[W])
    if 12 % W:
        raise ValueError(f"W = {W} does not divide 12")
    return 12 - 12 // W


def accel_units(f_w: dict, scale: int = 4096) -> dict:
    """Integer units of saved time from measured accelerations F_W (Sec. 5.B):
    round(scale (1 - 1/F_W)), at least 0 (a packing slower than W = 1 saves nothing)."""
    return {int(W): max(0, int(round(scale * (1.0 - 1.0 / float(f))))) for W, f in f_w.items()}


def accel_target(nl: int, w_max: int, frac: float, units: dict | None = None) -> float:
    """Required saved work of an inner kernel: the fraction `frac` of what
    packing every pair at w_max saves."""
    return frac * nl * saved_units(w_max, units)


def prune_accel(options: list[dict[int, PairOption]], w_desc: list[int], frac: float,
                units: dict | None = None) -> list[int]:
    """Sec. 6 pruning under the throughput constraint F_kernel = frac.

    Starting from the maximum packing, the outcome with the highest distortion
    (lowest l among equals) drops to the next smaller allowed W as long as the
    inner kernel still saves at least accel_target() units of MFMA work after
    the drop; it stops before the first drop that would break the constraint
    and once the highest remaining distortion is 0 (nothing to gain). With
    W in {1, 2}, frac is the fraction of subblock products that stay packed.
    An unavailable option (D >= D_UNAVAILABLE) drops whatever the constraint:
    its product could not be formed. units: measured saved-time units per W
    (see saved_units); None counts nominal MFMA work.
    """
    nl = len(options)
    level = [0] * nl
    d = [options[l][w_desc[0]].d for l in range(nl)]
    saved = sum(saved_units(w_desc[0], units) for _ in range(nl))
    target = accel_target(nl, w_desc[0], frac, units)
    while True:
        cand = [l for l in range(nl) if level[l] < len(w_desc) - 1]
        if not cand:
            break
        lstar = cand[0]
        for l in cand[1:]:
            if d[l] > d[lstar]:
                lstar = l
        if not d[lstar] > 0.0:
            break
        w_now, w_next = w_desc[level[lstar]], w_desc[level[lstar] + 1]
        after = saved - saved_units(w_now, units) + saved_units(w_next, units)
        if after < target and d[lstar] < D_UNAVAILABLE:
            break
        saved = after
        level[lstar] += 1
        d[lstar] = options[lstar][w_desc[level[lstar]]].d
    return [w_desc[level[l]] for l in range(nl)]


def signal_term(L_eff: int, sa: BlockStats, sb: BlockStats) -> float:
    """L_eff s_a^2 s_b^2, one term of the Sec. 6 budget."""
    s_a, s_b = sa.sigma, sb.sigma
    return (float(L_eff) * (s_a * s_a)) * (s_b * s_b)


def kernel_budget(signal_terms: list[float], snr_db: float) -> float:
    """Sec. 6: D_kernel = 10^(-0.1 S) sum_l L s_a^2 s_b^2 (exactly rounded sum)."""
    return 10.0 ** (-snr_db / 10.0) * exact_sum(signal_terms)


def prune(options: list[dict[int, PairOption]], w_desc: list[int], d_kernel: float) -> list[int]:
    """Sec. 6 top-down pruning of one inner kernel.

    options[l][W] is the pair option of subblock l at packing W; w_desc lists
    the allowed packings in descending order. Returns the chosen W per l.
    Removal goes on while the sum exceeds the budget or an unavailable option
    (D >= D_UNAVAILABLE, always the largest) is still current.
    """
    nl = len(options)
    level = [0] * nl
    d = [options[l][w_desc[0]].d for l in range(nl)]
    while True:
        cand = [l for l in range(nl) if level[l] < len(w_desc) - 1]
        if not cand:
            break
        lstar = cand[0]
        for l in cand[1:]:
            if d[l] > d[lstar]:
                lstar = l
        if not exact_sum(d) > d_kernel and d[lstar] < D_UNAVAILABLE:
            break
        level[lstar] += 1
        d[lstar] = options[lstar][w_desc[level[lstar]]].d
    return [w_desc[level[l]] for l in range(nl)]
