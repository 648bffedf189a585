"""Quantization / combined noise model and companders (oracle; test infrastructure only).

* Prop. 2, eq. (19): E{(rho - rho_hat)^2} = L[(s_a s_nb)^2 + (s_b s_na)^2 + (s_na s_nb)^2],
  with s_n = 1 / (c sqrt 12) the rounding noise of a compander c (Sec. 4.C).
* eq. (20): expected SNR = 10 log10(L s_a^2 s_b^2 / noise).
* eq. (21): combined noise D_W = eq. (19) + [s(R_max, W) / (c_A c_B)]^2.
* eq. (24): c_tot = L max|A| max|B| / R_max, so that c_A c_B = 1 / c_tot (eq. 17).
* Prop. 4, eq. (26): c_A* = sqrt(s_b / (s_a c_tot)), c_B* = sqrt(s_a / (s_b c_tot)).
* Prop. 3, eqs. (22)-(25): the general admissible companders for a target SNR.

Reading of the garbled eqs. (23), (27), (33): as printed they carry
((12 s)^2 + 1) / (144 s_a^2 s_b^2 c_tot^-2) -- not invariant under A -> tA -- and
drop the 1/L of the representation term. Evaluating eq. (21) at the eq. (26)
companders instead gives the normalised noise

    NSR(R) = c_tot / (6 s_a s_b) + c_tot^2 / (144 s_a^2 s_b^2)
             + s^2 c_tot^2 / (L s_a^2 s_b^2),

which the oracle uses for the expected SNR of Prop. 4 (eq. 27 read this way),
and the matching D_QvR = 12 s_a^2 s_b^2 / 10^(S/10) - c_tot^2 (1 + (12 s)^2 / L) / 12
for Prop. 3. Every expression below is evaluated in the order written, so a
GPU implementation can reproduce it operation for operation.
"""
from __future__ import annotations

import math

SQRT12 = math.sqrt(12.0)


def sigma_nu(c: float) -> float:
    """Rounding-noise standard deviation of a compander c (Sec. 4.C)."""
    return 1.0 / (c * SQRT12)


def quant_noise_eq19(L: float, s_a: float, s_b: float, c_a: float, c_b: float) -> float:
    """Eq. (19): expected quantization-noise power of one output."""
    na = sigma_nu(c_a)
    nb = sigma_nu(c_b)
    return L * ((s_a * nb) * (s_a * nb) + (s_b * na) * (s_b * na) + (na * nb) * (na * nb))


def snr_eq20(L: float, s_a: float, s_b: float, noise: float) -> float:
    """Eq. (20): expected SNR in dB of an output with the given noise power."""
    return 10.0 * math.log10(L * (s_a * s_b) * (s_a * s_b) / noise)


def combined_noise_eq21(L: float, s_a: float, s_b: float, c_a: float, c_b: float,
                        s_rep: float) -> float:
    """Eq. (21): D_W = eq. (19) + (s(R_max, W) / (c_A c_B))^2."""
    rep = s_rep / (c_a * c_b)
    return quant_noise_eq19(L, s_a, s_b, c_a, c_b) + rep * rep


def c_tot_eq24(L: float, amax_a: float, amax_b: float, r_max: float) -> float:
    """Eq. (24): c_tot = L max|A| max|B| / R_max."""
    return (L * amax_a * amax_b) / r_max


def companders_eq26(s_a: float, s_b: float, c_tot: float) -> tuple[float, float]:
    """Prop. 4, eq. (26): the minimum-error companders."""
    return math.sqrt(s_b / (s_a * c_tot)), math.sqrt(s_a / (s_b * c_tot))


def nsr_prop4(L: float, s_a: float, s_b: float, c_tot: float, s_rep: float) -> float:
    """Normalised noise at the eq. (26) companders (eq. 27 under the reading above)."""
    ss = s_a * s_b
    t1 = c_tot / (6.0 * ss)
    t2 = (c_tot * c_tot) / (144.0 * (ss * ss))
    t3 = ((s_rep * s_rep) * (c_tot * c_tot)) / (L * (ss * ss))
    return (t1 + t2) + t3


def d_qvr_eq23(L: float, s_a: float, s_b: float, snr_db: float, c_tot: float,
               s_rep: float) -> float:
    """Eq. (23) under the reading above: quantization-versus-representation term."""
    ss = s_a * s_b
    return 12.0 * ss * ss / 10.0 ** (0.1 * snr_db) - c_tot * c_tot * (1.0 + (12.0 * s_rep) ** 2 / L) / 12.0


def companders_eq22(L: float, s_a: float, s_b: float, snr_db: float, c_tot: float,
                    s_rep: float, sign: int = +1) -> tuple[float, float] | None:
    """Prop. 3, eq. (22): companders reaching snr_db, or None when eq. (25) fails."""
    d = d_qvr_eq23(L, s_a, s_b, snr_db, c_tot, s_rep)
    disc = d * d - 4.0 * s_a * s_a * s_b * s_b * c_tot * c_tot
    if d < 2.0 * s_a * s_b * c_tot or disc < 0.0:     # eq. (25)
        return None
    root = math.sqrt(d + sign * math.sqrt(disc))
    c_a = root / (math.sqrt(2.0) * s_a * c_tot)
    c_b = math.sqrt(2.0) * s_a / root
    return c_a, c_b
