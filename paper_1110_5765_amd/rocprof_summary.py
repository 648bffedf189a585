"""Summaries of rocprofv3 CSV output (``-f csv``) as short text.

    python -m paper_1110_5765_amd.rocprof_summary kernels DIR
        per-kernel dispatch statistics from *kernel_stats.csv
    python -m paper_1110_5765_amd.rocprof_summary counters DIR
        mean counter value per dispatch, per kernel, from *counter_collection.csv
    python -m paper_1110_5765_amd.rocprof_summary traffic FETCH WRITE PROBE_FETCH PROBE_WRITE \\
            --probe-bytes N --kernel REGEX --key KEY --out FILE [--sources P ...]
        HBM bytes per launch of one kernel: FETCH_SIZE and WRITE_SIZE (KiB per
        dispatch) scaled by what the same counters read for a plain copy kernel
        that reads and writes N bytes, written as JSON together with a hash of
        the kernel's sources (a changed kernel invalidates the figure).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import statistics
import sys


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits[0]


def kernel_stats(d: str) -> list[dict]:
    with open(_find(d, "kernel_stats.csv"), newline="") as f:
        return list(csv.DictReader(f))


def counter_means(d: str) -> dict:
    """{(kernel, counter): (mean value per dispatch, dispatches)}"""
    acc: dict = {}
    with open(_find(d, "counter_collection.csv"), newline="") as f:
        for row in csv.DictReader(f):
            key = (row["Kernel_Name"], row["Counter_Name"])
            acc.setdefault(key, {}).setdefault(row["Dispatch_Id"], 0.0)
            acc[key][row["Dispatch_Id"]] += float(row["Counter_Value"])
    return {k: (statistics.fmean(v.values()), len(v)) for k, v in acc.items()}


def _short(name: str, n: int = 72) -> str:
    return name if len(name) <= n else name[: n - 3] + "..."


def cmd_kernels(a) -> None:
    rows = kernel_stats(a.dir)
    print(f"{'kernel':72s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'total_ms':>10s}")
    for r in rows:
        print(f"{_short(r['Name']):72s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.1f} "
              f"{float(r['MinNs']) / 1e3:10.1f} {float(r['MaxNs']) / 1e3:10.1f} "
              f"{float(r['TotalDurationNs']) / 1e6:10.3f}")


def cmd_counters(a) -> None:
    for (k, c), (v, n) in sorted(counter_means(a.dir).items()):
        print(f"{_short(k):72s} {c:24s} dispatches={n:4d} mean={v:.6g}")


def _one(d: str, counter: str, regex: str) -> float:
    vals = [(v, n) for (k, c), (v, n) in counter_means(d).items() if c == counter and re.search(regex, k)]
    if len(vals) != 1:
        raise SystemExit(f"{counter}: expected one kernel matching {regex!r} in {d}, found {len(vals)}")
    return vals[0][0]


def cmd_traffic(a) -> None:
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    fetch = _one(a.fetch, "FETCH_SIZE", a.kernel)
    write = _one(a.write, "WRITE_SIZE", a.kernel)
    pf = _one(a.probe_fetch, "FETCH_SIZE", a.probe_kernel)
    pw = _one(a.probe_write, "WRITE_SIZE", a.probe_kernel)
    f_scale = a.probe_bytes / (pf * 1024.0)
    w_scale = a.probe_bytes / (pw * 1024.0)
    total = fetch * 1024.0 * f_scale + write * 1024.0 * w_scale
    h = hashlib.sha256()
    for p in a.sources:
        with open(os.path.join(root, p), "rb") as f:
            h.update(f.read())
    out = {}
    if os.path.exists(a.out):
        with open(a.out) as f:
            out = json.load(f)
    src = h.hexdigest()[:16]
    if out.get("source_hash") != src:
        out = {"source_hash": src, "sources": a.sources, "workloads": {}}
    out["workloads"][a.key] = {
        "kernel_regex": a.kernel, "fetch_kib": fetch, "write_kib": write,
        "fetch_scale": f_scale, "write_scale": w_scale, "hbm_bytes_per_launch": total,
        "probe_bytes": a.probe_bytes, "probe_fetch_kib": pf, "probe_write_kib": pw}
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out["workloads"][a.key]))


def main(argv=None) -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels"); k.add_argument("dir"); k.set_defaults(fn=cmd_kernels)
    c = sub.add_parser("counters"); c.add_argument("dir"); c.set_defaults(fn=cmd_counters)
    t = sub.add_parser("traffic")
    for n in ("fetch", "write", "probe_fetch", "probe_write"):
        t.add_argument(n)
    t.add_argument("--probe-bytes", type=float, required=True)
    t.add_argument("--probe-kernel", default="elementwise")
    t.add_argument("--kernel", required=True)
    t.add_argument("--key", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--sources", nargs="+", default=[])
    t.set_defaults(fn=cmd_traffic)
    a = ap.parse_args(argv)
    a.fn(a)


if __name__ == "__main__":
    main(sys.argv[1:])
