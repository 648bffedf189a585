"""Benchmark of the throughput-distortion GEMM on one MI355X.

One step = the whole hot path on one batch of synthetic input resident in HBM:
block statistics of A and B, the per-pair plan with inner-kernel pruning, and
the fused compand / pack / packed-product / unpack / reverse-compand kernel.
Workload (default): the 4096^3 throughput-distortion sweep point with i.i.d.
N(0, 1) FP64 inputs, L = 128, symmetric packing, S_kernel = 40 dB for every
inner kernel, W in {1, 2, 4}. The calibration table s(R, W) is measured on the
GPU before timing (offline, as the paper prescribes).

Prints ONE JSON line on stdout. Metric: effective GFLOP/s = 2 M N K / step
time, at the stated output SNR against the plain FP64 product.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import pathlib
import sys
import time

ROOT = pathlib.Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

PEAK_F64_TFLOPS = 78.6      # MI355X dense FP64 matrix peak
PEAK_F32_TFLOPS = 157.3
HBM_GBS = 8000.0

FUSED_SOURCES = ["paper_1110_5765_amd/csrc/fused.hip", "paper_1110_5765_amd/csrc/mfma.h",
                 "paper_1110_5765_amd/csrc/common.h"]


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def source_hash(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        h.update((ROOT / p).read_bytes())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--dist", default="gaussian", choices=["gaussian", "laplace", "random_range"])
    ap.add_argument("--L", type=int, default=128)
    ap.add_argument("--form", default="sym", choices=["sym", "asym"])
    ap.add_argument("--snr", type=float, default=40.0)
    ap.add_argument("--w", default="1,2,4")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-tiles", type=int, default=16)
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only run a plain copy kernel of known size (for counter scaling)")
    return ap.parse_args()


def calibrate_gpu(td, torch, L, form, prec, ws):
    """s(R, W) measured on the GPU path (Sec. 4.B protocol), W in ws."""
    import workloads
    from numpy import asarray
    ua, ub = workloads.calib_uniforms(L)
    dev_a = torch.from_numpy(ua).cuda()
    dev_b = torch.from_numpy(ub).cuda()
    q_max = (1 << 18) if prec == "f64" else (1 << 10)
    qs, k = [], 0
    while True:
        q = int(round(2.0 ** (k / 8)))
        if q > q_max:
            break
        if not qs or q != qs[-1]:
            qs.append(q)
        k += 1
    table = {}
    r0 = None
    for W in ws:
        r, m, s = td.tdgemm_calibrate(L, W, form, prec, qs, dev_a, dev_b)
        r0 = r if r0 is None else r0
        table[W] = s
    return td.DeviceCalib(asarray(r0), table), r0, table


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the sharded design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.traffic_probe:
        n = 1 << 27                       # 1 GiB of float64 read, 1 GiB written
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.add(x, 0.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"traffic_probe_bytes_read": n * 8, "bytes_written": n * 8}))
        return

    import workloads
    from paper_1110_5765_amd import tdgemm as td

    ws_allowed = tuple(int(x) for x in args.w.split(","))
    n = args.n
    log(f"[bench] workload {args.dist} {n}^3 FP64, L={args.L}, {args.form}, S={args.snr} dB, W={ws_allowed}")
    A, B = workloads.sweep(args.dist, n=n)
    Ad = torch.from_numpy(A).cuda()
    Bd = torch.from_numpy(B).cuda()
    torch.cuda.synchronize()

    t0 = time.time()
    calib, calib_r, calib_s = calibrate_gpu(td, torch, args.L, args.form, "f64", [w for w in ws_allowed if w > 1])
    log(f"[bench] GPU calibration of s(R, W): {time.time() - t0:.1f} s, {len(calib_r)} grid points")

    desc = td.make_desc(Ad, Bd, L=args.L, form=args.form, ctrl="snr", snr_db=args.snr, w_allowed=ws_allowed)
    ws = torch.empty(td.tdgemm_workspace_size(desc), dtype=torch.uint8, device="cuda")
    C = torch.empty((n, n), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        plan = td.tdgemm_plan(desc, Ad, Bd, calib, ws)
        if ev is not None:
            ev[1].record(stream)
        td.tdgemm_gemm(plan, Ad, Bd, C, fused=1)
        if ev is not None:
            ev[2].record(stream)
        return plan

    for _ in range(args.warmup):
        plan = step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for k in range(args.steps):
        plan = step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    plan_ms = [e[0].elapsed_time(e[1]) for e in evs]
    fused_ms = [e[1].elapsed_time(e[2]) for e in evs]
    step_ms = wall * 1e3 / args.steps
    flops = 2.0 * n * n * n
    gflops = flops / (step_ms * 1e-3) / 1e9
    log(f"[bench] step {step_ms:.3f} ms (plan+stats {np.mean(plan_ms):.3f} ms, fused {np.mean(fused_ms):.3f} ms)"
        f" -> {gflops:.1f} effective GFLOP/s")

    # accuracy and plan summary (outside the timed region)
    sa, sb, pairs, budget = td.tdgemm_plan_export(plan)
    wh = {int(w): int((pairs["w"] == w).sum()) for w in (1, 2, 4)}
    ref = torch.matmul(Ad, Bd)
    err = C - ref
    snr = 10.0 * math.log10(float((ref * ref).sum()) / float((err * err).sum()))
    L = args.L
    exec_flops = float(sum(2.0 * L * L * L / w * cnt for w, cnt in wh.items()))
    fused_avg = float(np.mean(fused_ms))
    achieved_tf = exec_flops / (fused_avg * 1e-3) / 1e12
    log(f"[bench] SNR vs FP64 {snr:.2f} dB, W histogram {wh}, executed MFMA {achieved_tf:.2f} TFLOP/s in the fused kernel")

    # plain GEMMs on the same GPU
    plain = {}
    if not args.no_plain:
        def time_it(fn, reps=10):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - s0) / reps
        t64 = time_it(lambda: torch.matmul(Ad, Bd, out=ref))
        A32, B32 = Ad.float(), Bd.float()
        C32 = torch.empty((n, n), dtype=torch.float32, device="cuda")
        t32 = time_it(lambda: torch.matmul(A32, B32, out=C32))
        e32 = C32.double() - ref
        snr32 = 10.0 * math.log10(float((ref * ref).sum()) / float((e32 * e32).sum()))
        plain = {"plain_fp64_gflops": round(flops / t64 / 1e9, 1), "plain_fp64_ms": round(t64 * 1e3, 3),
                 "plain_fp32_gflops": round(flops / t32 / 1e9, 1), "plain_fp32_ms": round(t32 * 1e3, 3),
                 "plain_fp32_snr_db": round(snr32, 2)}
        log(f"[bench] plain FP64 {plain['plain_fp64_gflops']} GFLOP/s, plain FP32 {plain['plain_fp32_gflops']}"
            f" GFLOP/s at {snr32:.1f} dB")

    # traffic from committed counter measurements, if they match the current kernel
    traffic = None
    tpath = ROOT / "profiles" / "fused_traffic.json"
    if tpath.exists():
        try:
            t = json.loads(tpath.read_text())
            key = f"{args.dist}_{n}_L{L}_{args.form}_S{args.snr:g}"
            if t.get("source_hash") == source_hash(FUSED_SOURCES) and key in t.get("workloads", {}):
                traffic = t["workloads"][key]["hbm_bytes_per_launch"]
        except (ValueError, KeyError):
            traffic = None

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(A, B, args)
        log(f"[bench] oracle on the host: {cpu['value']:.4f} GFLOP/s ({cpu['sample']})")

    out = {
        "metric": "effective GFLOP/s at fixed output SNR vs plain FP64 GEMM; % of FP64 MFMA peak",
        "value": round(gflops, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"throughput-distortion sweep point: C = A B, M = N = K = {n}, A and B i.i.d. "
                               f"{'N(0,1)' if args.dist == 'gaussian' else args.dist} FP64, L = {L}, "
                               f"{args.form} packing, S_kernel = {args.snr:g} dB, W in {list(ws_allowed)}",
                   "M": n, "N": n, "K": n, "L": L, "form": args.form, "snr_target_db": args.snr,
                   "parallelism": "single GPU"},
        "snr_db": round(snr, 2),
        "pct_fp64_mfma_peak": round(100.0 * gflops / (PEAK_F64_TFLOPS * 1e3), 1),
        "w_histogram": wh,
        "plan_ms": round(float(np.mean(plan_ms)), 4),
        "fused_ms": round(fused_avg, 4),
        **plain,
        "roofline": {"bound": "mfma", "kernel": "k_fused (FP64 16x16x4 MFMA)",
                     "achieved": round(achieved_tf, 2), "peak": PEAK_F64_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved_tf / PEAK_F64_TFLOPS, 4), "traffic": traffic},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(A, B, args):
    """The oracle on the host: statistics of every block plus the full pipeline on a
    few inner kernels, extrapolated to the whole product. Its calibration table
    comes from the oracle's own measurement (untimed, like the GPU's)."""
    import numpy as np
    import workloads
    from oracle import blocks as bk
    from oracle import calibration as cal
    from oracle import pipeline as pl

    from threadpoolctl import threadpool_limits

    L = args.L
    n = A.shape[0]
    with threadpool_limits(limits=1):
        return _cpu_baseline(A, B, args, L, n)


def _cpu_baseline(A, B, args, L, n):
    import numpy as np
    import workloads
    from oracle import blocks as bk
    from oracle import calibration as cal
    from oracle import pipeline as pl

    ua, ub = workloads.calib_uniforms(L)
    tabs = {W: cal.calibrate(L, W, args.form, "f64", ua, ub, q_max=1 << 18)[0]
            for W in (int(x) for x in args.w.split(",")) if W > 1}
    cfg = pl.Config(L=L, form=args.form, prec="f64", ctrl="snr", snr_db=args.snr,
                    w_allowed=tuple(int(x) for x in args.w.split(",")))
    nb = bk.n_blocks(n, L)
    rng = np.random.default_rng(0)
    tiles = [(int(i), int(j)) for i, j in rng.integers(0, nb, (args.cpu_tiles, 2))]
    t0 = time.perf_counter()
    plan = pl.make_plan(A, B, cfg, tabs, tiles=tiles)
    t1 = time.perf_counter()
    pl.run(A, B, cfg, tabs, tiles=tiles, plan=plan)
    t2 = time.perf_counter()
    # make_plan = statistics of all blocks + options/pruning for the sampled tiles
    total = (t1 - t0) + (t2 - t1) * (nb * nb) / len(tiles)
    return {"value": 2.0 * n ** 3 / total / 1e9, "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "sample": f"block statistics of all of A and B plus plan and pipeline for {len(tiles)} of "
                      f"{nb * nb} inner kernels ({t2 - t0:.1f} s), extrapolated to all inner kernels"}


if __name__ == "__main__":
    main()
