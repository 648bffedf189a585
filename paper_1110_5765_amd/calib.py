"""Calibration table s(R, W) measured on the GPU path (Sec. 4.B), as a DeviceCalib.

The grid is R = L q^2 over integer ranges q on a geometric grid (8 points per
octave) up to 2^18 (FP64 packing) or 2^10 (FP32 packing); the measurement
itself runs in tdgemm_calibrate. The uniform draws it maps to integer inputs
come from the seeded workload generators.

Sec. 5.B builds this table once, offline. A measured table can be kept in a
versioned JSON file (write_table / read_table, every value as an exact
hexadecimal float) and reused by device_table(..., cache=path) as long as its
block size, form, precision, packings and grid match.
"""
from __future__ import annotations

import json
import os

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


TABLE_VERSION = 1


def write_table(path: str, L: int, form: str, prec: str, r, table: dict) -> None:
    """Store r[k] and s_W[k] (W in table) exactly; +inf marks unusable points."""
    doc = {"format": "tdgemm-calibration", "version": TABLE_VERSION, "L": int(L), "form": form,
           "prec": prec, "r": [float(x).hex() for x in np.asarray(r, dtype=np.float64)],
           "s": {str(int(W)): [float(x).hex() for x in np.asarray(v, dtype=np.float64)]
                 for W, v in sorted(table.items())}}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f)
    os.replace(tmp, path)


def read_table(path: str, L: int, form: str, prec: str, ws):
    """(r, {W: s}) from a file written by write_table; ValueError if it does not
    hold this block size, form, precision and every packing in ws, or if its
    grid is not the one q_grid(prec) gives."""
    with open(path) as f:
        doc = json.load(f)
    if doc.get("format") != "tdgemm-calibration" or doc.get("version") != TABLE_VERSION:
        raise ValueError(f"{path}: not a version {TABLE_VERSION} calibration table")
    if (doc["L"], doc["form"], doc["prec"]) != (int(L), form, prec):
        raise ValueError(f"{path}: table for L={doc['L']} {doc['form']} {doc['prec']}, "
                         f"wanted L={L} {form} {prec}")
    r = np.array([float.fromhex(x) for x in doc["r"]])
    want = np.array([float(L) * q * q for q in q_grid(prec)])
    if r.shape != want.shape or not np.array_equal(r, want):
        raise ValueError(f"{path}: calibration grid differs from this version's")
    table = {}
    for W in ws:
        v = doc["s"].get(str(int(W)))
        if v is None or len(v) != r.size:
            raise ValueError(f"{path}: no s(R, {W}) of {r.size} points")
        table[int(W)] = np.array([float.fromhex(x) for x in v])
    return r, table


def device_table(L: int, form: str, prec: str, ws=(2, 4), device="cuda", cache: str | None = None):
    """(DeviceCalib, r, {W: s}) for packings ws. With `cache`, a matching table
    stored there is used instead of measuring, and a new measurement is stored."""
    if cache is not None and os.path.exists(cache):
        try:
            r, table = read_table(cache, L, form, prec, ws)
            return td.DeviceCalib(r, table, device=device), r, table
        except ValueError:
            pass                              # stale or other settings: measure again
    import workloads
    ua, ub = workloads.calib_uniforms(L)
    dev_a = torch.from_numpy(ua).to(device)
    dev_b = torch.from_numpy(ub).to(device)
    table, r0 = {}, None
    for W in ws:
        r, m, s = td.tdgemm_calibrate(L, W, form, prec, q_grid(prec), dev_a, dev_b)
        r0 = r if r0 is None else r0
        table[W] = s
    if cache is not None:
        write_table(cache, L, form, prec, r0, table)
    return td.DeviceCalib(np.asarray(r0), table, device=device), r0, table
