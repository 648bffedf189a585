"""Representation-noise measurement s(R_max, W), m(R_max, W) (oracle; test infrastructure only).

Sec. 4.B: integer inputs (so c_A = c_B = 1 and companding loses nothing),
uniform in [-max|A|, max|A|] and [-max|B|, max|B|], five random instances per
setting; z from eq. (15) for R_max = L max|A| max|B| (eq. 17 with c = 1); the
packed product is unpacked and compared with the conventional product. Eq.
(18) gives the mean error m and the RMSE s.

Readings taken:

* The paper fixes max|A| = 22 and sweeps max|B| over 1..63 to cover its
  R_max range. The range needed here is far wider, and the eq. (26) companders
  make Q_A / Q_B = (max|A|/s_a) / (max|B|/s_b), about 1 for i.i.d. blocks, so
  the sweep uses max|A| = max|B| = q over a geometric grid of integers q,
  giving R_max = L q^2. ``measure`` also takes a separate max|B| (R_max =
  L max|A| max|B|), the paper's own protocol.
* Eq. (18) prints (1/L^2) times a Frobenius norm; s is read as the per-output
  RMSE sqrt(mean e^2) and m as the mean error, in integer (index) units, over
  all outputs of all instances. Both sums are exactly rounded.
* The reference is the exact integer product (int64); for the paper's
  settings it coincides with the W = 1 product in the same data type.
* The random numbers are inputs: u_a, u_b are uniform [0, 1) draws, shape
  (instances, L, L), mapped to integers by floor(u (2q + 1)) - q; the same
  draws serve every grid point.
"""
from __future__ import annotations

import math

import numpy as np

from . import packing as pk
from .control import CalibTable
from .exactsum import exact_sum


def int_inputs(u: np.ndarray, q: int) -> np.ndarray:
    """Uniform integers in {-q, ..., q} from uniform [0, 1) draws."""
    return np.floor(np.asarray(u, dtype=np.float64) * float(2 * q + 1)) - float(q)


def q_grid(q_max: int = 1 << 20, steps_per_octave: int = 8) -> list[int]:
    """Geometric grid of integer ranges q = round(2^(k / steps)), deduplicated."""
    out, k = [], 0
    while True:
        q = int(round(2.0 ** (k / steps_per_octave)))
        if q > q_max:
            break
        if not out or q != out[-1]:
            out.append(q)
        k += 1
    return out


def measure(L: int, W: int, form: str, prec: str, q: int, u_a: np.ndarray, u_b: np.ndarray,
            u_safe: float = 50.0, q_b: int | None = None) -> tuple[float, float, float]:
    """(R_max, m, s) of eq. (18) for the packed product with max|A| = q and
    max|B| = q_b (default q), over all instances: R_max = L q q_b (eq. 17 with
    c = 1), m the mean and s the root mean square of the unpacked-minus-exact
    errors over every output of every instance."""
    q_b = q if q_b is None else q_b
    r_max = float(L) * float(q) * float(q_b)
    p = pk.packing_exponent(r_max, u_safe)
    errs = []
    for t in range(u_a.shape[0]):
        a = int_inputs(u_a[t], q)
        b = int_inputs(u_b[t], q_b)
        exact = a.astype(np.int64) @ b.astype(np.int64)
        dt = pk.DTYPES[prec]
        qa, qb = a.astype(dt), b.astype(dt)
        if form == "sym":
            rbar = pk.packed_product(pk.pack_sym_a(qa, W, p, prec), pk.pack_sym_b(qb, W, p, prec), prec)
            r = pk.unpack_sym(rbar, p, prec)
        else:
            rbar = pk.packed_product(pk.pack_asym_a(qa, W, p, prec), qb, prec)
            r = pk.unpack_asym(rbar, W, p, prec)
        with np.errstate(invalid="ignore", over="ignore"):
            e = np.asarray(r, dtype=np.float64) - exact.astype(np.float64)
        errs.append(e.ravel())
    e = np.concatenate(errs)
    n = e.size
    if not np.all(np.isfinite(e)):
        return r_max, float("nan"), float("inf")
    m = exact_sum(e.tolist()) / n
    s = math.sqrt(exact_sum((e * e).tolist()) / n)
    return r_max, m, s


def calibrate(L: int, W: int, form: str, prec: str, u_a: np.ndarray, u_b: np.ndarray,
              q_max: int = 1 << 20, u_safe: float = 50.0):
    """Sweep the grid; returns (CalibTable, list of (R, m, s) rows)."""
    rows = [measure(L, W, form, prec, q, u_a, u_b, u_safe) for q in q_grid(q_max)]
    r = np.array([x[0] for x in rows])
    s = np.array([x[2] for x in rows])
    return CalibTable(r, s), rows
