"""Calibration tables s(R, W) computed by the oracle (cached per process).

Used by the CPU pin tests and, as an input handed to both sides, by the GPU
parity tests: the plan of the GPU library and the oracle's plan then start
from the same table. Nothing here comes from the GPU path.
"""
from __future__ import annotations

import functools

import numpy as np

from oracle import calibration as cal
from workloads import calib_uniforms

# Widest q range that matters per precision (beyond it every setting is catastrophic).
Q_MAX = {"f64": 1 << 18, "f32": 1 << 10}


@functools.lru_cache(maxsize=None)
def table(L: int, W: int, form: str, prec: str):
    ua, ub = calib_uniforms(L)
    tab, rows = cal.calibrate(L, W, form, prec, ua, ub, q_max=Q_MAX[prec])
    return tab


def tables(L: int, form: str, prec: str, ws=(2, 4)) -> dict:
    return {W: table(L, W, form, prec) for W in ws if W > 1}


def as_arrays(tab) -> tuple[np.ndarray, np.ndarray]:
    return np.asarray(tab.r, dtype=np.float64), np.asarray(tab.s, dtype=np.float64)
