"""Calibration table s(R, W) measured on the GPU path (Sec. 4.B), as a DeviceCalib.

The grid is R = L q^2 over integer ranges q on a geometric grid (8 points per
octave) up to 2^18 (FP64 packing) or 2^10 (FP32 packing); the measurement
itself runs in tdgemm_calibrate. The uniform draws it maps to integer inputs
come from the seeded workload generators.

Sec. 5.B builds this table once, offline, and keeps beside it the
acceleration F_W of every packing, also found by off-line timing on the
target: measure_accel() times the fused product with every pair at packing W
against every pair at W = 1 (the throughput control uses 1 - 1/F_W, as integer
units from accel_units()). A measured table can be kept in a versioned JSON
file (write_table / read_table, every value as an exact hexadecimal float) and
reused by device_table(..., cache=path) as long as its block size, form,
precision, packings and grid match.
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


TABLE_VERSION = 2


def write_table(path: str, L: int, form: str, prec: str, r, table: dict, accel: dict | None = None) -> None:
    """Store r[k] and s_W[k] (W in table) exactly; +inf marks unusable points.
    accel: measured F_W per packing, kept beside the table (optional)."""
    doc = {"format": "tdgemm-calibration", "version": TABLE_VERSION, "L": int(L), "form": form,
           "prec": prec, "r": [float(x).hex() for x in np.asarray(r, dtype=np.float64)],
           "s": {str(int(W)): [float(x).hex() for x in np.asarray(v, dtype=np.float64)]
                 for W, v in sorted(table.items())}}
    if accel:
        doc["accel"] = {str(int(W)): float(f).hex() for W, f in sorted(accel.items())}
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


def read_accel(path: str) -> dict | None:
    """Measured F_W stored beside a table by write_table, or None."""
    with open(path) as f:
        doc = json.load(f)
    acc = doc.get("accel")
    return None if acc is None else {int(W): float.fromhex(x) for W, x in acc.items()}


def accel_units(f_w: dict, scale: int = 4096) -> dict:
    """Integer saved-time units for tdgemm_desc.accel_units: round(scale (1 - 1/F_W)),
    at least 0 (a packing slower than W = 1 saves nothing)."""
    return {int(W): max(0, int(round(scale * (1.0 - 1.0 / float(f))))) for W, f in f_w.items()}


def measure_accel(L: int, form: str, prec: str, ws=(2, 4), n: int = 4096, reps: int = 10,
                  device="cuda") -> dict:
    """F_W (Sec. 5.B): the mean time of the fused product of an n x n x n problem
    with every pair at W = 1 over its time with every pair at packing W (FIXED
    control: the work of a pair depends on W only). Inputs are the seeded
    Gaussian sweep matrices (float32 for FP32 packing); plan kernels are not timed."""
    import workloads
    A, B = workloads.sweep("gaussian", n=n)
    dt = np.float64 if prec == "f64" else np.float32
    Ad = torch.from_numpy(A.astype(dt)).to(device)
    Bd = torch.from_numpy(B.astype(dt)).to(device)
    C = torch.empty((n, n), dtype=Ad.dtype, device=device)
    stream = torch.cuda.current_stream()
    times = {}
    for W in (1, *ws):
        desc = td.make_desc(Ad, Bd, L=L, form=form, prec=prec, ctrl="fixed", fixed_w=W,
                            fixed_rmax=float(2 ** 12))
        plan = td.tdgemm_plan(desc, Ad, Bd, None)
        for _ in range(3):
            td.tdgemm_gemm(plan, Ad, Bd, C, fused=1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            td.tdgemm_gemm(plan, Ad, Bd, C, fused=1)
        e1.record(stream)
        torch.cuda.synchronize()
        times[W] = e0.elapsed_time(e1) / reps
    return {W: times[1] / times[W] for W in ws}


def device_table(L: int, form: str, prec: str, ws=(2, 4), device="cuda", cache: str | None = None,
                 with_accel: bool = False):
    """(DeviceCalib, r, {W: s}) for packings ws. With `cache`, a matching table
    stored there is used instead of measuring, and a new measurement is stored.
    with_accel: F_W is measured too (or read from the cache) and attached to the
    DeviceCalib as .accel ({W: F_W}) and .units (accel_units of it)."""
    if cache is not None and os.path.exists(cache):
        try:
            r, table = read_table(cache, L, form, prec, ws)
            acc = read_accel(cache)
            if not with_accel or (acc is not None and all(W in acc for W in ws)):
                dev = td.DeviceCalib(r, table, device=device)
                if with_accel:
                    dev.accel, dev.units = acc, accel_units(acc)
                return dev, r, table
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
    acc = measure_accel(L, form, prec, ws, device=device) if with_accel else None
    if cache is not None:
        write_table(cache, L, form, prec, r0, table, acc)
    dev = td.DeviceCalib(np.asarray(r0), table, device=device)
    if with_accel:
        dev.accel, dev.units = acc, accel_units(acc)
    return dev, r0, table
