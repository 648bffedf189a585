"""Stored calibration tables (host logic, no GPU): exact round trip of s(R, W),
rejection of tables for other settings, and reuse through device_table's cache."""
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cal():
    from paper_1110_5765_amd import calib
    return calib


def _table(cal, L, prec, ws, seed=3):
    r = np.array([float(L) * q * q for q in cal.q_grid(prec)])
    rng = np.random.default_rng(seed)
    table = {}
    for W in ws:
        s = rng.random(r.size) * 10.0 ** rng.integers(-12, 3, r.size)
        s[: 5 + W] = 0.0
        s[-3:] = np.inf                      # points past the packing's exact range
        table[W] = s
    return r, table


def test_round_trip_is_exact(cal, tmp_path):
    for L, form, prec, ws in [(128, "sym", "f64", (2, 4)), (96, "asym", "f64", (2, 3)),
                              (64, "sym", "f32", (2,))]:
        r, table = _table(cal, L, prec, ws)
        p = str(tmp_path / f"t{L}{form}{prec}.json")
        cal.write_table(p, L, form, prec, r, table)
        r2, t2 = cal.read_table(p, L, form, prec, ws)
        assert r2.tobytes() == r.tobytes()
        for W in ws:
            assert t2[W].tobytes() == table[W].tobytes()


def test_rejects_other_settings(cal, tmp_path):
    r, table = _table(cal, 128, "f64", (2, 4))
    p = str(tmp_path / "t.json")
    cal.write_table(p, 128, "sym", "f64", r, table)
    for args in [(64, "sym", "f64", (2, 4)), (128, "asym", "f64", (2, 4)),
                 (128, "sym", "f32", (2, 4)), (128, "sym", "f64", (2, 3))]:
        with pytest.raises(ValueError):
            cal.read_table(p, *args)
    doc = json.load(open(p))
    bad = dict(doc, version=doc["version"] + 1)
    json.dump(bad, open(p, "w"))
    with pytest.raises(ValueError):
        cal.read_table(p, 128, "sym", "f64", (2, 4))
    bad = dict(doc, r=doc["r"][:-1])
    json.dump(bad, open(p, "w"))
    with pytest.raises(ValueError):
        cal.read_table(p, 128, "sym", "f64", (2, 4))


def test_cache_is_used_without_measuring(cal, tmp_path, monkeypatch):
    r, table = _table(cal, 128, "f64", (2, 4))
    p = str(tmp_path / "cache.json")
    cal.write_table(p, 128, "sym", "f64", r, table)

    def no_measure(*a, **k):
        raise AssertionError("a matching cached table must not be measured again")

    monkeypatch.setattr(cal.td, "tdgemm_calibrate", no_measure)
    dev, r2, t2 = cal.device_table(128, "sym", "f64", (2, 4), device="cpu", cache=p)
    assert r2.tobytes() == r.tobytes()
    s = dev.s.numpy().reshape(3, -1)
    assert s[0].tobytes() == table[2].tobytes() and s[2].tobytes() == table[4].tobytes()
    assert np.all(np.isinf(s[1]))             # W = 3 not in the table


def test_accel_round_trip_and_units(cal, tmp_path):
    """F_W kept beside the table (Sec. 5.B) round-trips exactly; the integer units
    of the throughput control are round(4096 (1 - 1/F_W)), at least 0."""
    r, table = _table(cal, 128, "f64", (2, 4))
    p = str(tmp_path / "t.json")
    acc = {2: 1.3312345678, 4: 1.9}
    cal.write_table(p, 128, "sym", "f64", r, table, acc)
    assert cal.read_accel(p) == acc
    cal.write_table(p, 128, "sym", "f64", r, table)
    assert cal.read_accel(p) is None
    assert cal.accel_units({2: 2.0, 3: 1.0, 4: 0.5}) == {2: 2048, 3: 0, 4: 0}
    assert cal.accel_units(acc) == {2: round(4096 * (1 - 1 / 1.3312345678)), 4: round(4096 * (1 - 1 / 1.9))}
