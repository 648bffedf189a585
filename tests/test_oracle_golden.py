"""Pins of the oracle against values the paper prints (fixtures in tests/golden/)."""
import pathlib

import numpy as np

from oracle.calibration import measure

GOLDEN = pathlib.Path(__file__).parent / "golden"


def _fixture(name):
    out = {}
    for line in (GOLDEN / name).read_text().splitlines():
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            out[k] = v
    return out


def test_sec4b_single_precision_symmetric_w2_error_bounds():
    """Sec. 4.B: FP32 symmetric W = 2 packing at R_max <= 320000 has |m| / R_max
    < 1e-6 and s / R_max < 4e-4 under the Sec. 4.B protocol (eq. 18 errors of the
    packed product of eqs. 6-10 against the exact integer product). Loose pin
    (see the fixture): s / R_max within an order of magnitude of the printed
    bound, the mean error negligible against s, and s > 0 (single precision is
    beyond the exact regime of Prop. 1 there)."""
    f = _fixture("sec4b_sp_sym_w2_bounds.txt")
    L, W = int(f["L"]), int(f["W"])
    qa, qb = int(f["max_a"]), int(f["max_b"])
    inst = int(f["instances"])
    rng = np.random.default_rng(20111)
    ua, ub = rng.random((inst, L, L)), rng.random((inst, L, L))
    r_max, m, s = measure(L, W, f["form"], f["prec"], qa, ua, ub, q_b=qb)
    assert r_max == float(L * qa * qb) and r_max <= 320000.0
    k = float(f["magnitude_factor"])
    assert s / r_max < k * float(f["s_over_rmax_below"]), (s, r_max)
    assert s / r_max > float(f["s_over_rmax_below"]) / k, (s, r_max)
    assert abs(m) < float(f["m_over_s_below"]) * s, (m, s)
    assert s > 0.0
