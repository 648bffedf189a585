"""Calibration table s(R, W) measured on the GPU path (Sec. 4.B), as a DeviceCalib.

The grid is R = L q^2 over integer ranges q on a geometric grid (8 points per
octave) up to 2^18 (FP64 packing) or 2^10 (FP32 packing); the measurement
itself runs in tdgemm_calibrate. The uniform draws it maps to integer inputs
come from the seeded workload generators.
"""
from __future__ import annotations

import numpy as np
import torch

from . import tdgemm as td


def q_grid(prec: str) -> list[int]:
    q_max = (1 << 18) if prec == "f64" else (1 << 10)
    qs, k = [], 0
    while True:
        q = int(round(2.0 ** (k / 8)))
        if q > q_max:
            return qs
        if not qs or q != qs[-1]:
            qs.append(q)
        k += 1


def device_table(L: int, form: str, prec: str, ws=(2, 4), device="cuda"):
    """(DeviceCalib, r, {W: s}) for packings ws."""
    import workloads
    ua, ub = workloads.calib_uniforms(L)
    dev_a = torch.from_numpy(ua).to(device)
    dev_b = torch.from_numpy(ub).to(device)
    table, r0 = {}, None
    for W in ws:
        r, m, s = td.tdgemm_calibrate(L, W, form, prec, q_grid(prec), dev_a, dev_b)
        r0 = r if r0 is None else r0
        table[W] = s
    return td.DeviceCalib(np.asarray(r0), table, device=device), r0, table
