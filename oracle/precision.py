"""INT8 / FP8 block-scaled form on the same rounded operands (oracle; test infrastructure only).

Remark 1 weighs computing the companded products with integer arithmetic
instead of floating-point packing. This module is the plain definition of that
form on the block structure of Sec. 2:

* Separable block scales (Sec. 3.A companding with a fixed range Q): one
  compander per L x L block, c = Q / max|X| (c = 0 for an all-zero block), so
  the rounded operands are shared by every pair a block is part of. The pair
  record is the separable option with W = 1 (nothing is packed).
* INT8: q = [[c x]] (round half to even) in [-Q, Q], Q <= 127.
* FP8: q = E4M3(c x), the OCP E4M3FN value nearest to c x (ties to even
  mantissa), saturating at the largest finite value 448; Q <= 448.
* Per pair (i, l, j): r = sum_k qA[m, k] qB[k, n]. For INT8 the sum is exact
  (int64). For FP8 each product of two E4M3 values is exact and so is their
  sum in float64 (at most 43 significant bits), rounded once to float32.
* Reverse companding (eq. 5) and the l-sum of eq. (2), in float32: inv32 =
  float32(1 / (c_A c_B)), and per output C = fma(float32(r), inv32, C) for l
  ascending from C = 0 -- one correctly rounded fused multiply-add per pair,
  i.e. an FMA chain over l (the paper fixes the rounding of neither step; one
  rounding per pair is the plainest). C is float32: the form accumulates in
  32-bit arithmetic.

E4M3FN (OCP 8-bit floating point, format E4M3): 1 sign bit, 4 exponent bits
with bias 7, 3 mantissa bits; exponent field 0 holds the subnormals m 2^-9;
the code S.1111.111 is NaN and there are no infinities, so the largest finite
magnitude is 1.75 * 2^8 = 448.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import blocks as bk
from . import control as ct
from .fmachain import fma_matmul
from .pipeline import Config

FORMATS = ("i8", "e4m3")
Q_LIMIT = {"i8": 127.0, "e4m3": 448.0}
E4M3_MAX = 448.0
E4M3_MIN_NORMAL = 2.0 ** -6
E4M3_SUBNORMAL_STEP = 2.0 ** -9


# ---------------------------------------------------------------------------
# E4M3FN codec

def e4m3_decode(code: int) -> float:
    """Value of an E4M3FN byte (NaN for S.1111.111)."""
    s = -1.0 if code & 0x80 else 1.0
    e = (code >> 3) & 0xF
    m = code & 0x7
    if e == 0xF and m == 0x7:
        return math.nan
    if e == 0:
        return s * m * E4M3_SUBNORMAL_STEP
    return s * (8 + m) * 2.0 ** (e - 10)


def e4m3_round(v: float) -> float:
    """Nearest E4M3FN value to v, ties to even mantissa, saturating at +-448.
    The sign of zero follows v."""
    a = abs(v)
    if a == 0.0:
        return math.copysign(0.0, v)
    if a >= E4M3_MAX:
        return math.copysign(E4M3_MAX, v)
    if a < E4M3_MIN_NORMAL:
        step = E4M3_SUBNORMAL_STEP
    else:
        e = math.frexp(a)[1] - 1           # a in [2^e, 2^(e+1))
        step = 2.0 ** (e - 3)
    q = float(np.rint(a / step)) * step    # a / step is exact (power-of-two step)
    return math.copysign(min(q, E4M3_MAX), v)


def e4m3_encode(v: float) -> int:
    """E4M3FN byte of a representable value (as returned by e4m3_round)."""
    s = 0x80 if math.copysign(1.0, v) < 0 else 0
    a = abs(v)
    if a == 0.0:
        return s
    if a < E4M3_MIN_NORMAL:
        m = a / E4M3_SUBNORMAL_STEP
        assert m == int(m) and 1 <= m <= 7
        return s | int(m)
    e = math.frexp(a)[1] - 1
    m = a / 2.0 ** (e - 3) - 8.0
    assert m == int(m) and 0 <= m <= 7 and -6 <= e <= 8
    return s | ((e + 7) << 3) | int(m)


# ---------------------------------------------------------------------------
# Plan records and quantized operands

def block_scaled_option(L_eff: int, sa: bk.BlockStats, sb: bk.BlockStats, q: float,
                        u_safe: float) -> ct.PairOption:
    """Separable companders c = Q / max|X| of a pair, W = 1 (no packing)."""
    if sa.amax == 0.0 or sb.amax == 0.0:
        return ct.option_zero(1, u_safe)
    return dataclasses.replace(ct.separable_option(2, L_eff, sa, sb, q, u_safe), W=1)


def block_scale(st: bk.BlockStats, q: float) -> float:
    """c = Q / max|X| of one block; 0 for an all-zero block."""
    return 0.0 if st.amax == 0.0 else q / st.amax


def quantize_block(x: np.ndarray, c: float, fmt: str) -> np.ndarray:
    """Rounded operands of one block, as float64 values (INT8: integers)."""
    v = np.asarray(x, dtype=np.float64) * c
    if fmt == "i8":
        return np.rint(v)
    if fmt == "e4m3":
        return np.vectorize(e4m3_round, otypes=[np.float64])(v)
    raise ValueError(fmt)


def codes(q: np.ndarray, fmt: str) -> np.ndarray:
    """Byte codes of rounded operands: two's-complement int8, or E4M3FN."""
    if fmt == "i8":
        return q.astype(np.int64).astype(np.int8).view(np.uint8)
    return np.vectorize(e4m3_encode, otypes=[np.uint8])(q)


@dataclasses.dataclass
class Result:
    stats_a: list
    stats_b: list
    scale_a: np.ndarray          # [nI][nL]
    scale_b: np.ndarray          # [nL][nJ]
    options: dict                # (i, j, l) -> PairOption
    qa: np.ndarray               # (nI L) x (nL L) rounded values, zero padded
    qb: np.ndarray               # (nL L) x (nJ L)
    products: dict               # (i, j, l) -> r (int64 for INT8, float32 for FP8)
    C: np.ndarray                # M x N float32


def run(A: np.ndarray, B: np.ndarray, L: int, fmt: str, q: float, u_safe: float = 50.0,
        keep_products: bool = True) -> Result:
    """The whole block-scaled product C = A B in the given format."""
    if fmt not in FORMATS:
        raise ValueError(fmt)
    if not (1.0 <= q <= Q_LIMIT[fmt]):
        raise ValueError(f"range {q} outside [1, {Q_LIMIT[fmt]}] for {fmt}")
    M, K = A.shape
    N = B.shape[1]
    nI, nL, nJ = bk.n_blocks(M, L), bk.n_blocks(K, L), bk.n_blocks(N, L)
    sa = bk.all_block_stats(A, L)
    sb = bk.all_block_stats(B, L)
    scale_a = np.array([[block_scale(sa[i][l], q) for l in range(nL)] for i in range(nI)])
    scale_b = np.array([[block_scale(sb[l][j], q) for j in range(nJ)] for l in range(nL)])
    qa = np.zeros((nI * L, nL * L))
    qb = np.zeros((nL * L, nJ * L))
    for i in range(nI):
        for l in range(nL):
            qa[i * L:(i + 1) * L, l * L:(l + 1) * L] = quantize_block(bk.block(A, i, l, L), scale_a[i, l], fmt)
    for l in range(nL):
        for j in range(nJ):
            qb[l * L:(l + 1) * L, j * L:(j + 1) * L] = quantize_block(bk.block(B, l, j, L), scale_b[l, j], fmt)
    options, products = {}, {}
    C = np.zeros((nI * L, nJ * L), dtype=np.float32)
    for i in range(nI):
        for j in range(nJ):
            rs = np.zeros((nL, L, L), dtype=np.float32)      # float32(r) per l
            invs = np.zeros(nL, dtype=np.float32)             # float32(1 / (c_A c_B)) per l
            for l in range(nL):
                L_eff = bk.valid_extent(K, l, L)
                o = block_scaled_option(L_eff, sa[i][l], sb[l][j], q, u_safe)
                options[(i, j, l)] = o
                a = qa[i * L:(i + 1) * L, l * L:(l + 1) * L]
                b = qb[l * L:(l + 1) * L, j * L:(j + 1) * L]
                if fmt == "i8":
                    r = a.astype(np.int64) @ b.astype(np.int64)
                    r32 = r.astype(np.float32)          # exact: |r| <= L Q^2 < 2^24
                else:
                    r = a @ b                           # exact in float64 (see header)
                    r32 = r.astype(np.float32)
                if keep_products:
                    products[(i, j, l)] = r if fmt == "i8" else r32
                rs[l] = r32
                invs[l] = np.float32(o.inv)
            # per output, the FMA chain over l ascending: row (r_0 .. r_nL-1) by column (inv_0 ..)
            rows = np.ascontiguousarray(rs.reshape(nL, L * L).T).reshape(L * L, 1, nL)
            cols = np.ascontiguousarray(np.broadcast_to(invs.reshape(1, nL, 1), (L * L, nL, 1)))
            C[i * L:(i + 1) * L, j * L:(j + 1) * L] = fma_matmul(rows, cols, "f32").reshape(L, L)
    return Result(sa, sb, scale_a, scale_b, options, qa, qb, products, C[:M, :N])


def exact_fp8_sums_fit(L: int) -> bool:
    """Bound behind the exact float64 sum of E4M3 products: products are
    multiples of 2^-18 below 448^2 < 2^18, so L of them need 36 + log2(L) bits."""
    return 36 + math.ceil(math.log2(L)) <= 53


def default_config(L: int = 128) -> Config:
    """Separable configuration the packed FP64 form uses on the same integers."""
    return Config(L=L, form="sym", prec="f64", ctrl="separable", fixed_w=2, sep_q=127.0)
