"""Shared helpers of the GPU parity tests: run the HIP path through the C-ABI and
the oracle on the same inputs, and compare."""
from __future__ import annotations

import sys

import numpy as np
import torch

from oracle import pipeline as pl
from tests.oracle_tables import tables


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def device_calib(td, L: int, form: str, prec: str, ws=(2, 4)):
    tabs = tables(L, form, prec, ws)
    r = tabs[ws[0]].r
    for W in ws:
        assert np.array_equal(tabs[W].r, r)
    return td.DeviceCalib(r, {W: tabs[W].s for W in ws}), tabs


def to_dev(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def oracle_cfg(L, form, prec, ctrl, snr_db, w_allowed, fixed_w, fixed_rmax, sep_q):
    return pl.Config(L=L, form=form, prec=prec, ctrl=ctrl, snr_db=snr_db, w_allowed=tuple(w_allowed),
                     fixed_w=fixed_w, fixed_rmax=fixed_rmax, sep_q=sep_q)


PAIR_FIELDS = ["c_a", "c_b", "inv", "d", "r_max", "s_rep", "q_a", "q_b"]


def compare_plan(gpu_pairs, gpu_budget, gpu_sa, gpu_sb, res, tiles):
    """Bit-exact comparison of statistics, pair records and budgets."""
    plan = res.plan
    nI, nL, nJ = plan.grid
    for i in range(nI):
        for l in range(nL):
            s, o = gpu_sa[i, l], plan.stats_a[i][l]
            assert (s["mn"], s["mx"], s["sumsq"], s["n"]) == (o.mn, o.mx, o.sumsq, o.n), ("A", i, l)
    for l in range(nL):
        for j in range(nJ):
            s, o = gpu_sb[l, j], plan.stats_b[l][j]
            assert (s["mn"], s["mx"], s["sumsq"], s["n"]) == (o.mn, o.mx, o.sumsq, o.n), ("B", l, j)
    for (i, j) in tiles:
        for l in range(nL):
            g, o = gpu_pairs[i, j, l], plan.chosen[(i, j, l)]
            assert int(g["w"]) == o.W and int(g["p"]) == o.p, (i, j, l, g, o)
            for f in PAIR_FIELDS:
                assert float(g[f]) == float(getattr(o, f)), (f, i, j, l, float(g[f]), getattr(o, f))
        if plan.cfg.ctrl == "snr":
            assert gpu_budget[i, j] == plan.budget[(i, j)]


def assert_elementwise(got, want, A, B, tol, what="C"):
    """|got - want| <= tol * (|A| |B|) element by element: the magnitude of the
    terms that eq. (2) sums bounds the rounding differences of any summation
    order (a zero row or column of A or B must then match exactly)."""
    bound = tol * (np.abs(np.asarray(A, dtype=np.float64)) @ np.abs(np.asarray(B, dtype=np.float64)))
    d = np.abs(np.asarray(got, dtype=np.float64) - np.asarray(want, dtype=np.float64))
    bad = ~(d <= bound)
    if bad.any():
        k = np.unravel_index(np.argmax(np.where(bad, d - bound, -np.inf)), d.shape)
        raise AssertionError(f"{what}: {int(bad.sum())} elements beyond tol {tol:g} x |A||B|; "
                             f"worst at {k}: |diff| {d[k]:.3e} > {bound[k]:.3e}")


def rel_err(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))
