"""Companding, packing, packed products and unpacking (oracle; test infrastructure only).

Follows Sec. 3 of the paper step by step, for one L x L subblock pair:

* eq. (3)   compand and round:      qa = [[c_A a]],  qb = [[c_B b]]
* eq. (6)   symmetric packing of A: Abar[m, nb] = sum_i z^i  qa[m, W nb + i]
* eq. (7)   symmetric packing of B: Bbar[mb, n] = sum_i z^-i qb[W mb + i, n]
* eq. (8)   symmetric packed product Rbar = Abar Bbar
* eqs. (9)-(10)  symmetric unpack:  u = [[rbar]],  r = u - z^-1 [[z u]]
* eq. (11)  asymmetric packing of W rows of A: Abar[mb, n] = sum_i z^i qa[W mb + i, n]
* eq. (12)  asymmetric packed product Rbar = Abar qB
* eqs. (13)-(14) asymmetric iterative unpack
* eq. (5)   reverse companding r_hat = r / (c_A c_B)
* Prop. 1, eqs. (15)-(17): packing coefficient bound, W_ef, R_max

Readings taken (the paper leaves these open):

* [[x]] is round-half-to-even (``numpy.rint``).
* z is a power of two, the largest one not above the bound of eq. (15):
  z = 2^-p with p = ceil(log2(2 R_safe + u_safe)); multiplying by z or z^-1 is
  then exact and eq. (10) subtracts an exact integer.
* The sums of eqs. (6), (7) and (11) are evaluated by Horner's rule from the
  highest slot down (acc = acc * z + q_i), so the order of the roundings that
  occur once a packed word no longer fits the mantissa is defined.
* In the garbled index of eq. (14), rbar_{mb+i} denotes the i-th peel of
  packed row mb; it yields r for row W mb + i.
* "prec" is the arithmetic the packed path runs in: 'f64' (dGEMM) or 'f32'
  (sGEMM). In 'f32', c_A is rounded to float32 and the block is multiplied in
  float32, as a single-precision kernel would.
"""
from __future__ import annotations

import math

import numpy as np

from .fmachain import fma_matmul

DTYPES = {"f64": np.float64, "f32": np.float32}
# Relative precision u_sys of eq. (16), read as machine epsilon (the
# conservative of the two usual meanings).
EPS = {"f64": 2.0 ** -52, "f32": 2.0 ** -23}
MANTISSA_BITS = {"f64": 53, "f32": 24}


def compand(X: np.ndarray, c: float, prec: str) -> np.ndarray:
    """Eq. (3): round-half-even of c * x, elementwise, in the packing precision."""
    dt = DTYPES[prec]
    return np.rint(dt(c) * np.asarray(X, dtype=dt)).astype(dt)


def decompand(r: np.ndarray, inv: float, prec: str) -> np.ndarray:
    """Eq. (5): r_hat = (c_A c_B)^-1 r, with inv = 1 / (c_A c_B) given."""
    dt = DTYPES[prec]
    return (np.asarray(r, dtype=dt) * dt(inv)).astype(dt)


def rmax_eq17(c_a: float, c_b: float, L: int, amax_a: float, amax_b: float) -> float:
    """Eq. (17): R_max = [[c_A c_B L max|A| max|B|]]."""
    return float(np.rint(c_a * c_b * L * amax_a * amax_b))


def z_bound_eq15(r_max: float, u_safe: float = 50.0) -> float:
    """Eq. (15): the largest z allowed for error-free packing."""
    return 1.0 / (2.0 * r_max + u_safe)


def packing_exponent(r_safe: float, u_safe: float = 50.0) -> int:
    """p = ceil(log2(2 R_safe + u_safe)), so z = 2^-p satisfies eq. (15).

    Computed exactly: 2 R_safe + u_safe is an integer below 2^53 and frexp is
    exact, so no logarithm is rounded.
    """
    v = 2.0 * r_safe + u_safe
    m, e = math.frexp(v)          # v = m 2^e, 0.5 <= m < 1
    return e - 1 if m == 0.5 else e


def w_ef_eq16(r_max: float, z: float, u_sys: float) -> int:
    """Eq. (16): W_ef = floor(log_z[(2 R_max + 1) u_sys] + 1)."""
    return int(math.floor(math.log((2.0 * r_max + 1.0) * u_sys) / math.log(z) + 1.0))


def _zpow(p: int, prec: str):
    dt = DTYPES[prec]
    return dt(math.ldexp(1.0, -p)), dt(math.ldexp(1.0, p))


def pack_sym_a(qa: np.ndarray, W: int, p: int, prec: str) -> np.ndarray:
    """Eq. (6): L x L/W block, W consecutive columns of qa per packed word."""
    L = qa.shape[1]
    z, _ = _zpow(p, prec)
    q = np.asarray(qa, dtype=DTYPES[prec]).reshape(qa.shape[0], L // W, W)
    acc = q[:, :, W - 1].copy()
    for i in range(W - 2, -1, -1):
        acc = acc * z + q[:, :, i]
    return acc


def pack_sym_b(qb: np.ndarray, W: int, p: int, prec: str) -> np.ndarray:
    """Eq. (7): L/W x L block, W consecutive rows of qb per packed word, weights z^-i."""
    L = qb.shape[0]
    _, zi = _zpow(p, prec)
    q = np.asarray(qb, dtype=DTYPES[prec]).reshape(L // W, W, qb.shape[1])
    acc = q[:, W - 1, :].copy()
    for i in range(W - 2, -1, -1):
        acc = acc * zi + q[:, i, :]
    return acc


def pack_asym_a(qa: np.ndarray, W: int, p: int, prec: str) -> np.ndarray:
    """Eq. (11): L/W x L block, W consecutive rows of qa per packed word."""
    L = qa.shape[0]
    z, _ = _zpow(p, prec)
    q = np.asarray(qa, dtype=DTYPES[prec]).reshape(L // W, W, qa.shape[1])
    acc = q[:, W - 1, :].copy()
    for i in range(W - 2, -1, -1):
        acc = acc * z + q[:, i, :]
    return acc


def packed_product(abar: np.ndarray, bbar: np.ndarray, prec: str) -> np.ndarray:
    """Eqs. (8) / (12): the ordinary product of the packed blocks, in prec.

    The paper runs an unchanged sGEMM/dGEMM subblock kernel on the packed data
    in its native representation and leaves the accumulation order open. The
    oracle takes the plainest order: every output is a chain of correctly
    rounded fused multiply-adds over the packed index, ascending, from 0.
    """
    return fma_matmul(abar, bbar, prec)


def unpack_sym(rbar: np.ndarray, p: int, prec: str) -> np.ndarray:
    """Eqs. (9)-(10): u = [[rbar]]; r = u - z^-1 [[z u]]."""
    z, zi = _zpow(p, prec)
    u = np.rint(rbar)
    return u - zi * np.rint(z * u)


def unpack_asym(rbar: np.ndarray, W: int, p: int, prec: str) -> np.ndarray:
    """Eqs. (13)-(14): peel W rows out of each packed row, highest weight first."""
    _, zi = _zpow(p, prec)
    Lw, N = rbar.shape
    out = np.zeros((Lw * W, N), dtype=rbar.dtype)
    t = rbar
    for i in range(W):
        r_i = np.rint(t)
        out[i::W, :] = r_i               # row W*mb + i
        if i < W - 1:
            t = zi * (t - r_i)
    return out


def exact_regime_sym(n: int, q_a: float, q_b: float, W: int, p: int, r_safe: float,
                     prec: str) -> bool:
    """Sufficient condition for the unpacked integers of eqs. (8)-(10) to be exact
    whatever the summation order of the packed product.

    Derived from Prop. 1 and eq. (8): every packed word must be representable,
    and the rounding error of an n-term dot product, at most
    gamma_n * T with T = sum |abar||bbar| <= n Q_A Q_B (sum z^i)(sum z^-h),
    plus the positive-power side outputs (W-d pairs at weight z^d) must stay
    below 1/2, while |r| <= R_safe < 2^(p-1) holds by the choice of p.
    """
    if W == 1:
        return False
    u = EPS[prec]
    mant = MANTISSA_BITS[prec]
    for q in (q_a, q_b):
        if math.ceil(math.log2(q + 1.0)) + (W - 1) * p > mant:
            return False
    z = 2.0 ** -p
    sz = sum(z ** i for i in range(W))
    szi = sum(z ** -i for i in range(W))
    T = n * q_a * q_b * sz * szi
    if n * u >= 1.0:
        return False
    gamma = n * u / (1.0 - n * u)
    side = sum(z ** d * (W - d) for d in range(1, W)) * n * q_a * q_b
    return (gamma * T + side) < 0.5 * (1.0 - 1e-9) and 2.0 * r_safe < 2.0 ** p


def exact_regime_asym(n: int, q_a: float, q_b: float, W: int, p: int, r_safe: float,
                      prec: str) -> bool:
    """Sufficient condition for exact integers from eqs. (11)-(14), any order.

    n = L terms per packed output; each peel of eq. (14) multiplies the
    remaining error by z^-1, so the last peel sees z^-(W-1) gamma_n T, and the
    lower slots contribute at most z R_safe / (1 - z) to each rounding.
    """
    if W == 1:
        return False
    u = EPS[prec]
    mant = MANTISSA_BITS[prec]
    if math.ceil(math.log2(q_a + 1.0)) + (W - 1) * p > mant:
        return False
    z = 2.0 ** -p
    T = n * q_a * q_b * sum(z ** i for i in range(W))
    if n * u >= 1.0:
        return False
    gamma = n * u / (1.0 - n * u)
    lower = z * r_safe / (1.0 - z)
    return (z ** -(W - 1) * gamma * T + lower) < 0.5 * (1.0 - 1e-9) and 2.0 * r_safe < 2.0 ** p
