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

--workload mlp: a 512 -> 1024 -> 1024 -> 10 perceptron, batch 4096, trained
for 200 SGD steps with every large product (forward and backward) through
the packed FP32 autograd layer, and the same training in plain FP32; ms per
step and both loss curves are reported.

--workload scatter: X^T X and X P for X = 2000 mean-removed uniform vectors of
10304 dimensions (float32) and a 10304 x 200 Gaussian P, packed FP64 at
S = 50, 40 and 20 dB against plain FP64 and FP32.

--workload sweep-table: the whole 4096^3 throughput-distortion sweep, S in
{60, 52, 44, 36, 28, 20} dB x {sym, asym} x L in {64, 96, 128} (W in {1, 2, 3} at
L = 96, {1, 2, 4} otherwise) x {Gaussian,
Laplace}, one line with every point (step time, effective GFLOP/s, SNR, W).

--workload fig7: throughput-controlled single-precision GEMM, 4032^3 with the
generic random-range inputs of Sec. 7, W in {1, 2}, F_kernel from 0 % to
100 % of the subblock products packed, symmetric and asymmetric forms.

--workload precision: the 8192^3 Laplace workload of the block-scaled form.

--workload pca2d: the 2D-PCA face-recognition application on synthetic 288 x 288
images (75 training, 90 test, d = 10): scatter-matrix and projection GEMMs with
FP32 packing at L = 96 at S = 40, 30, 20 dB, native and plain FP32, with the
recognition rate of each.
A step is tdgemm_plan (separable block scales) + tdgemm_compand (INT8 byte
operands) + the block-scaled tdgemm_gemm; the FP8 form, the packed FP64 form
at S = 30 and 40 dB and the plain FP64 / FP32 products on the same inputs are
timed beside it and reported in the same line.
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

FUSED_SOURCES = ["paper_1110_5765_amd/csrc/fused.h", "paper_1110_5765_amd/csrc/mfma.h",
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
    # 50 untimed steps bring the GPU to its steady clocks (after 5, the fused
    # kernel still ran 2-3 % slower); 100 timed steps of the default workload
    # take about 0.15 s
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-k-split", dest="k_split", action="store_false",
                    help="pca2d, scatter: one workgroup per inner kernel (no grouped l-sum)")
    ap.add_argument("--workload", default="sweep",
                    choices=["sweep", "precision", "mlp", "scatter", "sweep-table", "fig7", "pca2d", "accel"])
    ap.add_argument("--mlp-steps", type=int, default=200)
    ap.add_argument("--mlp-snr", type=float, default=20.0,
                    help="S_kernel of the packed FP32 products (W = 2 reaches about 20 dB)")
    ap.add_argument("--lr", type=float, default=0.1)
    ap.add_argument("--n", type=int, default=None, help="matrix size (4096 sweep, 8192 precision)")
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
    from paper_1110_5765_amd.calib import device_table
    return device_table(L, form, prec, tuple(ws))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: tdgemm runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the product would shard by inner kernel, one C panel per GPU)", file=sys.stderr)
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

    if args.workload == "precision":
        return run_precision(args)
    if args.workload == "mlp":
        return run_mlp(args)
    if args.workload == "scatter":
        return run_scatter(args)
    if args.workload == "sweep-table":
        return run_sweep_table(args)
    if args.workload == "pca2d":
        return run_pca2d(args)
    if args.workload == "fig7":
        return run_fig7(args)
    if args.workload == "accel":
        return run_accel(args)
    return run_sweep(args)


class _Joined:
    """A step's start event that is the previous step's end event: recording it
    again is a no-op, so back-to-back steps record one event between them."""

    def __init__(self, ev):
        self.ev = ev

    def record(self, stream=None):
        pass

    def elapsed_time(self, other):
        return self.ev.elapsed_time(other)


def timed_steps(torch, step, warmup, steps, phases):
    """W untimed steps, then exactly K timed steps between device synchronisations.
    step(ev) records events ev[0..phases] on the current stream between its phases;
    ev[0] of a step is the previous step's ev[phases] (each event recorded on the
    stream costs a few microseconds of idle GPU between the kernels it separates).
    Returns (ms per step by the host clock, [per-phase mean ms])."""
    import numpy as np
    for _ in range(warmup):
        step(None)
    torch.cuda.synchronize()
    evs = []
    for k in range(steps):
        first = torch.cuda.Event(enable_timing=True) if k == 0 else _Joined(evs[k - 1][phases])
        evs.append([first] + [torch.cuda.Event(enable_timing=True) for _ in range(phases)])
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ph = [float(np.mean([e[p].elapsed_time(e[p + 1]) for e in evs])) for p in range(phases)]
    return wall * 1e3 / steps, ph


def snr_of(torch, C, ref) -> float:
    err = C.double() - ref
    return 10.0 * math.log10(float((ref * ref).sum()) / float((err * err).sum()))


def time_plain(torch, Ad, Bd, ref, reps=10):
    """Plain FP64 and FP32 (on FP32-cast inputs) products on the same GPU."""
    def time_it(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - s0) / reps
    n, k = Ad.shape
    m = Bd.shape[1]
    flops = 2.0 * n * k * m
    C64 = torch.empty_like(ref)
    t64 = time_it(lambda: torch.matmul(Ad, Bd, out=C64))
    A32, B32 = Ad.float(), Bd.float()
    C32 = torch.empty((n, m), dtype=torch.float32, device="cuda")
    t32 = time_it(lambda: torch.matmul(A32, B32, out=C32))
    snr32 = snr_of(torch, C32, ref)
    return {"plain_fp64_gflops": round(flops / t64 / 1e9, 1), "plain_fp64_ms": round(t64 * 1e3, 3),
            "plain_fp32_gflops": round(flops / t32 / 1e9, 1), "plain_fp32_ms": round(t32 * 1e3, 3),
            "plain_fp32_snr_db": round(snr32, 2)}


def run_sweep(args):
    import numpy as np
    import torch

    import workloads
    from paper_1110_5765_amd import tdgemm as td

    ws_allowed = tuple(int(x) for x in args.w.split(","))
    n = args.n or 4096
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

    holder = {}

    def step(ev):
        if ev is not None:
            ev[0].record(stream)
        holder["plan"] = td.tdgemm_plan(desc, Ad, Bd, calib, ws)
        if ev is not None:
            ev[1].record(stream)
        td.tdgemm_gemm(holder["plan"], Ad, Bd, C, fused=1)
        if ev is not None:
            ev[2].record(stream)

    step_ms, (plan_avg, fused_avg) = timed_steps(torch, step, args.warmup, args.steps, 2)
    plan = holder["plan"]
    flops = 2.0 * n * n * n
    gflops = flops / (step_ms * 1e-3) / 1e9
    log(f"[bench] step {step_ms:.3f} ms (plan+stats {plan_avg:.3f} ms, fused {fused_avg:.3f} ms)"
        f" -> {gflops:.1f} effective GFLOP/s")

    # accuracy and plan summary (outside the timed region)
    sa, sb, pairs, budget = td.tdgemm_plan_export(plan)
    wh = {int(w): int((pairs["w"] == w).sum()) for w in ws_allowed}
    ref = torch.matmul(Ad, Bd)
    snr = snr_of(torch, C, ref)
    L = args.L
    exec_flops = float(sum(2.0 * L * L * L / w * cnt for w, cnt in wh.items()))
    achieved_tf = exec_flops / (fused_avg * 1e-3) / 1e12
    log(f"[bench] SNR vs FP64 {snr:.2f} dB, W histogram {wh}, executed MFMA {achieved_tf:.2f} TFLOP/s in the fused kernel")

    # plain GEMMs on the same GPU
    plain = {}
    if not args.no_plain:
        plain = time_plain(torch, Ad, Bd, ref)
        log(f"[bench] plain FP64 {plain['plain_fp64_gflops']} GFLOP/s, plain FP32 {plain['plain_fp32_gflops']}"
            f" GFLOP/s at {plain['plain_fp32_snr_db']} dB")

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
        log(f"[bench] oracle on the host ({cpu['cpu_model']}, {cpu['nproc']} CPUs): {cpu['value']:.4f} "
            f"GFLOP/s on {cpu['cores']} processes, {cpu['value_1thread']:.4f} GFLOP/s on one thread "
            f"({cpu['sample']})")

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
        "plan_ms": round(plan_avg, 4),
        "fused_ms": round(fused_avg, 4),
        **plain,
        "roofline": {"bound": "mfma", "kernel": "k_fused (FP64 16x16x4 MFMA)",
                     "achieved": round(achieved_tf, 2), "peak": PEAK_F64_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved_tf / PEAK_F64_TFLOPS, 4), "traffic": traffic},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def run_sweep_table(args):
    """Throughput-distortion sweep at 4096^3: every S, form, L and distribution."""
    import torch

    import workloads
    from paper_1110_5765_amd import tdgemm as td

    n = args.n or 4096
    flops = 2.0 * n ** 3
    stream = torch.cuda.current_stream()
    calibs = {}
    rows = []
    for dist in ("gaussian", "laplace"):
        A, B = workloads.sweep(dist, n=n)
        Ad = torch.from_numpy(A).cuda()
        Bd = torch.from_numpy(B).cuda()
        ref = torch.matmul(Ad, Bd)
        C = torch.empty((n, n), dtype=torch.float64, device="cuda")
        # packings a block size supports; L = 96 also with the whole set {1, 2, 3, 4} of Sec. 7
        for L, wset in ((64, (1, 2, 4)), (96, (1, 2, 3)), (96, (1, 2, 3, 4)), (128, (1, 2, 4))):
            for form in ("sym", "asym"):
                if (L, form) not in calibs:
                    calibs[(L, form)] = calibrate_gpu(td, torch, L, form, "f64",
                                                      [2, 3, 4] if L == 96 else [2, 4])[0]
                calib = calibs[(L, form)]
                for S in (60.0, 52.0, 44.0, 36.0, 28.0, 20.0):
                    desc = td.make_desc(Ad, Bd, L=L, form=form, ctrl="snr", snr_db=S, w_allowed=wset)
                    ws = torch.empty(td.tdgemm_workspace_size(desc), dtype=torch.uint8, device="cuda")
                    holder = {}

                    def step(ev, desc=desc, ws=ws, holder=holder):
                        if ev is not None:
                            ev[0].record(stream)
                        holder["plan"] = td.tdgemm_plan(desc, Ad, Bd, calib, ws)
                        td.tdgemm_gemm(holder["plan"], Ad, Bd, C, fused=1)
                        if ev is not None:
                            ev[1].record(stream)

                    # five warm-up steps: the clocks drop while the host evaluates a point
                    ms, _ = timed_steps(torch, step, 5, max(10, args.steps // 2), 1)
                    _, _, pairs, _ = td.tdgemm_plan_export(holder["plan"])
                    wh = {int(w): int((pairs["w"] == w).sum()) for w in wset}
                    snr = snr_of(torch, C, ref)
                    rows.append({"dist": dist, "L": L, "w_allowed": list(wset), "form": form,
                                 "snr_target_db": S, "ms": round(ms, 4),
                                 "gflops": round(flops / ms / 1e6, 1), "snr_db": round(snr, 2),
                                 "w_histogram": wh})
                    log(f"[bench] {dist:8s} L={L:3d} W<={max(wset)} {form:4s} S={S:4.0f}: {ms:7.3f} ms "
                        f"{flops / ms / 1e6:9.1f} GFLOP/s  SNR {snr:6.2f} dB  W {wh}")
                    del ws
        plain = time_plain(torch, Ad, Bd, ref)
        log(f"[bench] {dist}: plain FP64 {plain['plain_fp64_gflops']} GFLOP/s, plain FP32 "
            f"{plain['plain_fp32_gflops']} GFLOP/s at {plain['plain_fp32_snr_db']} dB")
        rows.append({"dist": dist, "plain": plain})
        del Ad, Bd, ref, C
    best = max((r for r in rows if "gflops" in r and r["snr_db"] >= 40.0), key=lambda r: r["gflops"])
    out = {
        "metric": "effective GFLOP/s at fixed output SNR vs plain FP64 GEMM; % of FP64 MFMA peak",
        "value": best["gflops"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": max(10, args.steps // 2),
        "warmup": 5,
        "ms_per_step": best["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"throughput-distortion sweep, M = N = K = {n}: best point with output SNR >= "
                               f"40 dB ({best['dist']}, L = {best['L']}, {best['form']}, S = "
                               f"{best['snr_target_db']:g} dB); all points in 'table'",
                   "parallelism": "single GPU"},
        "table": rows,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_fig7(args):
    """Throughput control sweep (F_kernel = 0 .. 100 %), FP32 packing, W in {1, 2}."""
    import torch

    import workloads
    from paper_1110_5765_amd import tdgemm as td

    n = args.n or 4032
    L = 64
    A = workloads.random_range((n, n), workloads.SEEDS["random_range"][0], L=L).astype("float32")
    B = workloads.random_range((n, n), workloads.SEEDS["random_range"][1], L=L).astype("float32")
    Ad = torch.from_numpy(A).cuda()
    Bd = torch.from_numpy(B).cuda()
    ref = torch.matmul(Ad.double(), Bd.double())
    flops = 2.0 * n ** 3
    stream = torch.cuda.current_stream()
    C = torch.empty((n, n), dtype=torch.float32, device="cuda")
    rows = []
    for form in ("sym", "asym"):
        calib = calibrate_gpu(td, torch, L, form, "f32", [2])[0]
        for k in range(11):
            F = k / 10.0
            desc = td.make_desc(Ad, Bd, L=L, form=form, prec="f32", ctrl="accel", accel=F, w_allowed=(1, 2))
            ws = torch.empty(td.tdgemm_workspace_size(desc), dtype=torch.uint8, device="cuda")
            holder = {}

            def step(ev, desc=desc, ws=ws, holder=holder, calib=calib):
                if ev is not None:
                    ev[0].record(stream)
                holder["plan"] = td.tdgemm_plan(desc, Ad, Bd, calib, ws)
                td.tdgemm_gemm(holder["plan"], Ad, Bd, C, fused=1)
                if ev is not None:
                    ev[1].record(stream)

            ms, _ = timed_steps(torch, step, 5, max(5, args.steps // 2), 1)
            _, _, pairs, _ = td.tdgemm_plan_export(holder["plan"])
            packed = float((pairs["w"] == 2).mean())
            snr = snr_of(torch, C, ref)
            rows.append({"form": form, "F_kernel": F, "packed_fraction": round(packed, 4), "ms": round(ms, 4),
                         "gflops": round(flops / ms / 1e6, 1), "snr_db": round(snr, 2)})
            log(f"[bench] fig7 {form:4s} F={F:3.1f}: packed {packed:6.1%}  {ms:7.3f} ms  "
                f"{flops / ms / 1e6:9.1f} GFLOP/s  SNR {snr:7.2f} dB")
    plain = time_plain(torch, Ad.double(), Bd.double(), ref)
    log(f"[bench] fig7 plain FP64 {plain['plain_fp64_gflops']} GFLOP/s, plain FP32 {plain['plain_fp32_gflops']} "
        f"GFLOP/s at {plain['plain_fp32_snr_db']} dB")
    full = {r["form"]: r for r in rows if r["F_kernel"] == 1.0}
    out = {
        "metric": "effective GFLOP/s at fixed output SNR vs plain FP64 GEMM; % of FP64 MFMA peak",
        "value": full["sym"]["gflops"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": max(5, args.steps // 2),
        "warmup": 5,
        "ms_per_step": full["sym"]["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"throughput control: {n}^3 float32 random-range inputs, FP32 packing, L = {L}, "
                               f"W in [1, 2], F_kernel = 100 % (sym); all points in 'table'",
                   "parallelism": "single GPU"},
        "snr_db": full["sym"]["snr_db"],
        "snr_gap_sym_minus_asym_db": round(full["sym"]["snr_db"] - full["asym"]["snr_db"], 2),
        "table": rows,
        **plain,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_accel(args):
    """Throughput control with W in {1, 2, 4} (4096^3 Gaussian FP64, L = 128): F_W
    measured on the GPU (Sec. 5.B) and F_kernel from 0 to 100 %, pruned with the
    measured saved-time units and with the nominal MFMA-work units."""
    import torch

    import workloads
    from paper_1110_5765_amd import calib as cb
    from paper_1110_5765_amd import tdgemm as td

    n = args.n or 4096
    L, form, ws_allowed = args.L, args.form, (1, 2, 4)
    A, B = workloads.sweep(args.dist, n=n)
    Ad = torch.from_numpy(A).cuda()
    Bd = torch.from_numpy(B).cuda()
    ref = torch.matmul(Ad, Bd)
    calib, _, _ = cb.device_table(L, form, "f64", (2, 4), with_accel=True)
    log(f"[bench] accel: measured F_W {calib.accel}, saved-time units {calib.units}")
    flops = 2.0 * n ** 3
    stream = torch.cuda.current_stream()
    C = torch.empty((n, n), dtype=torch.float64, device="cuda")
    rows = []
    for kind, units in (("measured", calib.units), ("nominal", None)):
        for F in (0.0, 0.25, 0.5, 0.75, 1.0):
            desc = td.make_desc(Ad, Bd, L=L, form=form, ctrl="accel", accel=F, w_allowed=ws_allowed,
                                accel_units=units)
            ws = torch.empty(td.tdgemm_workspace_size(desc), dtype=torch.uint8, device="cuda")
            holder = {}

            def step(ev, desc=desc, ws=ws, holder=holder):
                if ev is not None:
                    ev[0].record(stream)
                holder["plan"] = td.tdgemm_plan(desc, Ad, Bd, calib, ws)
                td.tdgemm_gemm(holder["plan"], Ad, Bd, C, fused=1)
                if ev is not None:
                    ev[1].record(stream)

            ms, _ = timed_steps(torch, step, 5, max(5, args.steps // 2), 1)
            _, _, pairs, _ = td.tdgemm_plan_export(holder["plan"])
            wh = {int(w): int((pairs["w"] == w).sum()) for w in ws_allowed}
            snr = snr_of(torch, C, ref)
            rows.append({"units": kind, "F_kernel": F, "ms": round(ms, 4), "gflops": round(flops / ms / 1e6, 1),
                         "snr_db": round(snr, 2), "w_histogram": wh})
            log(f"[bench] accel {kind:8s} F={F:4.2f}: {ms:7.3f} ms  {flops / ms / 1e6:9.1f} GFLOP/s  "
                f"SNR {snr:6.2f} dB  W {wh}")
    main = next(r for r in rows if r["units"] == "measured" and r["F_kernel"] == 1.0)
    out = {
        "metric": "effective GFLOP/s at fixed output SNR vs plain FP64 GEMM; % of FP64 MFMA peak",
        "value": main["gflops"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": max(5, args.steps // 2),
        "warmup": 5,
        "ms_per_step": main["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"throughput control: {n}^3 {args.dist} FP64, L = {L}, {form}, W in [1, 2, 4], "
                               f"measured F_W, F_kernel = 100 % (all points in 'table')",
                   "parallelism": "single GPU"},
        "accel_measured": {str(k): round(v, 4) for k, v in calib.accel.items()},
        "accel_units": {str(k): v for k, v in calib.units.items()},
        "snr_db": main["snr_db"],
        "table": rows,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_precision(args):
    """8192^3 Laplace: the block-scaled INT8 form timed as the step, FP8, packed FP64
    at S = 30 and 40 dB and the plain products beside it."""
    import torch

    import workloads
    from paper_1110_5765_amd import tdgemm as td

    n = args.n or 8192
    L = 128
    log(f"[bench] precision workload: Laplace(1) {n}^3 FP64, L = {L}, block-scaled INT8 / FP8 "
        f"vs packed FP64")
    A, B = workloads.precision(n)
    Ad = torch.from_numpy(A).cuda()
    Bd = torch.from_numpy(B).cuda()
    ref = torch.matmul(Ad, Bd)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    flops = 2.0 * n * n * n
    forms = {}
    for fmt, q in (("i8", 127.0), ("e4m3", 448.0)):
        desc = td.make_desc(Ad, Bd, L=L, prec=fmt, ctrl="separable", fixed_w=1, sep_q=q)
        ws = torch.empty(td.tdgemm_workspace_size(desc), dtype=torch.uint8, device="cuda")
        sh = td.block_scaled_shapes(td.tdgemm_plan(desc, Ad, Bd, None, ws))
        qA = torch.empty(sh["qA"], dtype=torch.uint8, device="cuda")
        qB = torch.empty(sh["qB"], dtype=torch.uint8, device="cuda")
        Cf = torch.empty((n, n), dtype=torch.float32, device="cuda")

        def step(ev, desc=desc, ws=ws, qA=qA, qB=qB, Cf=Cf):
            if ev is not None:
                ev[0].record(stream)
            plan = td.tdgemm_plan(desc, Ad, Bd, None, ws)
            if ev is not None:
                ev[1].record(stream)
            td.tdgemm_compand(plan, Ad, Bd, qA, qB)
            if ev is not None:
                ev[2].record(stream)
            td.tdgemm_gemm(plan, qA, qB, Cf, fused=1)
            if ev is not None:
                ev[3].record(stream)

        step_ms, (plan_ms, quant_ms, gemm_ms) = timed_steps(torch, step, args.warmup, args.steps, 3)
        snr = snr_of(torch, Cf, ref)
        forms[fmt] = {"step_ms": round(step_ms, 4), "gflops": round(flops / step_ms / 1e6, 1),
                      "snr_db": round(snr, 2), "plan_ms": round(plan_ms, 4),
                      "quant_ms": round(quant_ms, 4), "gemm_ms": round(gemm_ms, 4), "q": q}
        log(f"[bench] {fmt}: step {step_ms:.3f} ms (plan {plan_ms:.3f}, quantize {quant_ms:.3f}, "
            f"product {gemm_ms:.3f}) -> {flops / step_ms / 1e6:.1f} effective GFLOP/s at {snr:.2f} dB")
        del qA, qB, Cf, ws

    calib, _, _ = calibrate_gpu(td, torch, L, "sym", "f64", [2, 4])
    packed = {}
    C64 = torch.empty((n, n), dtype=torch.float64, device="cuda")
    for S in (30.0, 40.0):
        desc = td.make_desc(Ad, Bd, L=L, form="sym", ctrl="snr", snr_db=S, w_allowed=(1, 2, 4))
        ws = torch.empty(td.tdgemm_workspace_size(desc), dtype=torch.uint8, device="cuda")
        holder = {}

        def step(ev, desc=desc, ws=ws, holder=holder):
            if ev is not None:
                ev[0].record(stream)
            holder["plan"] = td.tdgemm_plan(desc, Ad, Bd, calib, ws)
            td.tdgemm_gemm(holder["plan"], Ad, Bd, C64, fused=1)
            if ev is not None:
                ev[1].record(stream)

        step_ms, _ = timed_steps(torch, step, 1, max(3, args.steps // 4), 1)
        _, _, pairs, _ = td.tdgemm_plan_export(holder["plan"])
        wh = {int(w): int((pairs["w"] == w).sum()) for w in (1, 2, 4)}
        snr = snr_of(torch, C64, ref)
        packed[f"S{S:g}"] = {"step_ms": round(step_ms, 3), "gflops": round(flops / step_ms / 1e6, 1),
                             "snr_db": round(snr, 2), "w_histogram": wh}
        log(f"[bench] packed FP64 sym L={L} S={S:g}: step {step_ms:.3f} ms -> {flops / step_ms / 1e6:.1f} "
            f"effective GFLOP/s at {snr:.2f} dB, W {wh}")
        del ws
    del C64
    plain = {} if args.no_plain else time_plain(torch, Ad, Bd, ref, reps=5)
    if plain:
        log(f"[bench] plain FP64 {plain['plain_fp64_gflops']} GFLOP/s, plain FP32 {plain['plain_fp32_gflops']}"
            f" GFLOP/s at {plain['plain_fp32_snr_db']} dB")
    cpu = None
    if not args.no_cpu_baseline:
        cpu = precision_cpu_baseline(A, B)
        log(f"[bench] oracle on the host: {cpu['value']:.4f} GFLOP/s ({cpu['sample']})")
    i8 = forms["i8"]
    tops = flops / (i8["gemm_ms"] * 1e-3) / 1e12
    out = {
        "metric": "effective GFLOP/s at fixed output SNR vs plain FP64 GEMM; % of FP64 MFMA peak",
        "value": i8["gflops"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": i8["step_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic",
        "config": {"workload": f"precision form: C = A B, M = N = K = {n}, A and B i.i.d. Laplace(1) FP64, "
                               f"L = {L}, separable block scales, INT8 (Q = 127) on the INT8 matrix cores",
                   "M": n, "N": n, "K": n, "L": L, "parallelism": "single GPU"},
        "snr_db": i8["snr_db"],
        "forms": forms,
        "packed_fp64": packed,
        **plain,
        "roofline": {"bound": "mfma", "kernel": "k_gemm8 (INT8 16x16x64 MFMA)", "achieved": round(tops, 1),
                     "peak": 5000.0, "unit": "TOP/s", "frac": round(tops / 5000.0, 4), "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


# untimed training steps before each timed run of the perceptron: with 3 (or 50) the first
# variant timed still ran about 25 % slower (clocks rising, first launches)
MLP_WARMUP = 200


def run_mlp(args):
    """Perceptron training with packed products (autograd layer) against plain FP32."""
    import numpy as np
    import torch

    import workloads
    from paper_1110_5765_amd import autograd
    from paper_1110_5765_amd import tdgemm as td
    from paper_1110_5765_amd.calib import device_table

    Ws, bs, xs, ys = workloads.mlp()
    L = args.L if args.L in (64, 128) else 64
    calib, _, _ = device_table(L, args.form, "f32", (2,))
    cfg = autograd.TDConfig(L=L, form=args.form, prec="f32", ctrl="snr", snr_db=args.mlp_snr,
                            w_allowed=(1, 2), min_dim=2 * L)
    tdc = autograd.TDContext(cfg, calib)
    # the same layer with its products in the INT8 block-scaled form (Remark 1)
    tdc8 = autograd.TDContext(autograd.TDConfig(L=128, prec="i8", ctrl="separable", sep_q=127.0,
                                                min_dim=128), None)
    X = torch.from_numpy(xs).cuda()
    Y = torch.from_numpy(ys).cuda()
    nsteps = args.mlp_steps
    log(f"[bench] MLP 512-1024-1024-10, batch {xs.shape[1]}, {nsteps} SGD steps (lr {args.lr}), "
        f"packed FP32 {args.form} L={L} S={args.mlp_snr:g} dB vs plain FP32")

    def make(packed):
        params = []
        for W, b in zip(Ws, bs):
            params.append((torch.from_numpy(W.copy()).cuda().requires_grad_(),
                           torch.from_numpy(b.copy()).cuda().requires_grad_()))
        return params

    def forward(params, x, packed):
        h = x
        for k, (W, b) in enumerate(params):
            if packed:
                h = autograd.TDLinearFn.apply(h, W, b, tdc8 if packed == "i8" else tdc)
            else:
                h = h @ W + b
            if k + 1 < len(params):
                h = torch.relu(h)
        return h

    def train(packed):
        params = make(packed)
        losses = []

        def one(k):
            x, y = X[k % X.shape[0]], Y[k % Y.shape[0]]
            loss = torch.nn.functional.cross_entropy(forward(params, x, packed), y)
            for W, b in params:
                W.grad = b.grad = None
            loss.backward()
            with torch.no_grad():
                for W, b in params:
                    W -= args.lr * W.grad
                    b -= args.lr * b.grad
            return loss

        for k in range(MLP_WARMUP):              # warm-up on a copy of the start
            one(k)
        params = make(packed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ls = [one(k) for k in range(nsteps)]
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / nsteps
        losses = [float(v) for v in ls]
        return ms, losses

    calls0 = tdc.calls
    ms_p, loss_p = train(True)
    packed_calls = (tdc.calls - calls0) / (nsteps + MLP_WARMUP)
    ms_q, loss_q = train(False)
    ms_8, loss_8 = train("i8")
    # distortion of one packed product of the trained shape (forward of layer 2)
    h = torch.randn(xs.shape[1], 1024, device="cuda")
    W2 = torch.from_numpy(Ws[1]).cuda()
    Cp = tdc.matmul(h, W2)
    _, _, pairs, _ = td.tdgemm_plan_export(tdc.last_plan)
    wh = {int(w): int((pairs["w"] == w).sum()) for w in (1, 2)}
    ref = (h.double() @ W2.double())
    err = Cp.double() - ref
    snr = 10.0 * math.log10(float((ref * ref).sum()) / float((err * err).sum()))
    flops = 0.0
    B = xs.shape[1]
    sizes = [W.shape for W in Ws]
    for k, (fi, fo) in enumerate(sizes):
        flops += 2.0 * B * fi * fo * (3 if k > 0 else 2)        # forward, dW (+ dX past layer 1)
    gap = max(abs(a - b) for a, b in zip(loss_p, loss_q))
    gap8 = max(abs(a - b) for a, b in zip(loss_8, loss_q))
    C8 = tdc8.matmul(h, W2)
    err8 = C8.double() - ref
    snr8 = 10.0 * math.log10(float((ref * ref).sum()) / float((err8 * err8).sum()))
    log(f"[bench] packed {ms_p:.3f} ms/step ({packed_calls:.0f} packed products per step), plain "
        f"{ms_q:.3f} ms/step; loss packed {loss_p[0]:.4f} -> {loss_p[-1]:.4f}, plain {loss_q[0]:.4f} -> "
        f"{loss_q[-1]:.4f}, max gap {gap:.4f}; layer-2 product SNR {snr:.1f} dB, W {wh}")
    log(f"[bench] INT8 block-scaled products: {ms_8:.3f} ms/step ({ms_q / ms_8:.2f}x the plain step); loss "
        f"{loss_8[0]:.4f} -> {loss_8[-1]:.4f}, max gap to plain {gap8:.4f}; layer-2 product SNR {snr8:.1f} dB")
    out = {
        "metric": "effective GFLOP/s at fixed output SNR vs plain FP64 GEMM; % of FP64 MFMA peak",
        "value": round(flops / ms_p / 1e6, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": nsteps,
        "warmup": MLP_WARMUP,
        "ms_per_step": round(ms_p, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"MLP 512-1024-1024-10, batch {B}, SGD lr {args.lr}, cross-entropy, packed "
                               f"FP32 {args.form} products (L = {L}, S = {args.mlp_snr:g} dB, W in [1, 2])",
                   "steps": nsteps, "parallelism": "single GPU"},
        "plain_fp32_ms_per_step": round(ms_q, 4),
        "plain_fp32_gflops": round(flops / ms_q / 1e6, 1),
        "loss_packed": [round(v, 5) for v in loss_p[:: max(1, nsteps // 20)]] + [round(loss_p[-1], 5)],
        "loss_plain": [round(v, 5) for v in loss_q[:: max(1, nsteps // 20)]] + [round(loss_q[-1], 5)],
        "max_loss_gap": round(gap, 5),
        "product_snr_db": round(snr, 2),
        "product_w_histogram": wh,
        "int8_block_scaled_ms_per_step": round(ms_8, 4),
        "int8_block_scaled_gflops": round(flops / ms_8 / 1e6, 1),
        "loss_int8_block_scaled": [round(v, 5) for v in loss_8[:: max(1, nsteps // 20)]] + [round(loss_8[-1], 5)],
        "max_loss_gap_int8": round(gap8, 5),
        "int8_product_snr_db": round(snr8, 2),
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


PCA_WARMUP = 100


def run_pca2d(args):
    """2D-PCA face recognition (Sec. 8.A) on the synthetic 288 x 288 images: the
    image scatter matrix G = sum_j A_j^T A_j (one GEMM over the stacked training
    images), the projections Y = A X of training and test images onto the d = 10
    leading eigenvectors of G, and nearest-neighbour matching. Every GEMM runs
    through the library (FP32 inputs and packing, L = 96, W in {1, 2}); the
    eigendecomposition (once per training set) and the matching are plain torch."""
    import torch

    import workloads
    from paper_1110_5765_amd import tdgemm as td

    L, d, size = 96, 10, 288
    tr, ltr, te, lte = workloads.faces()
    mu = tr.mean(0)
    Sd = torch.from_numpy((tr - mu).reshape(-1, size)).cuda()     # stacked training images
    Td = torch.from_numpy((te - mu).reshape(-1, size)).cuda()     # stacked test images
    n_tr, n_te = tr.shape[0], te.shape[0]
    calib = calibrate_gpu(td, torch, L, args.form, "f32", [2])[0]
    stream = torch.cuda.current_stream()
    shapes = {"G": (Sd.t(), Sd), "Yset": (Sd, None), "Ytest": (Td, None)}
    flops = 2.0 * (size * size * Sd.shape[0] + (Sd.shape[0] + Td.shape[0]) * size * d)
    log(f"[bench] 2D-PCA: {n_tr} training and {n_te} test images of {size} x {size}, d = {d}; "
        f"GEMMs G ({size}x{Sd.shape[0]} by {Sd.shape[0]}x{size}) and projections ({Sd.shape[0]} / "
        f"{Td.shape[0]} x {size} by {size} x {d}), FP32 packing {args.form} L = {L}, "
        f"k_split {'auto' if args.k_split else 1}")

    def gemm(A, B, snr, ws_cache):
        if snr is None:
            return torch.matmul(A, B)
        ks = td.auto_k_split(A.shape[0], B.shape[1], A.shape[1], L, "f32") if args.k_split else 1
        desc = td.make_desc(A, B, L=L, form=args.form, prec="f32", ctrl="snr", snr_db=snr, w_allowed=(1, 2),
                            k_split=ks)
        key = (A.shape, B.shape, A.stride(), B.stride(), ks)
        if key not in ws_cache:
            ws_cache[key] = torch.empty(td.tdgemm_workspace_size(desc), dtype=torch.uint8, device="cuda")
        plan = td.tdgemm_plan(desc, A, B, calib, ws_cache[key])
        C = torch.empty((A.shape[0], B.shape[1]), dtype=torch.float32, device="cuda")
        td.tdgemm_gemm(plan, A, B, C, fused=1)
        return C

    def pipeline(snr, ws_cache, X=None):
        G = gemm(Sd.t(), Sd, snr, ws_cache)
        if X is None:
            _, V = torch.linalg.eigh(G.double())
            X = V[:, -d:].flip(1).float().contiguous()
        Ys = gemm(Sd, X, snr, ws_cache)
        Yt = gemm(Td, X, snr, ws_cache)
        return G, X, Ys, Yt

    def recognise(Ys, Yt):
        dist = torch.cdist(Yt.reshape(n_te, -1).double(), Ys.reshape(n_tr, -1).double())
        return ltr[dist.argmin(1).cpu().numpy()]

    G64 = torch.matmul(Sd.t().double(), Sd.double())
    rows = []
    for snr in (None, math.inf, 40.0, 30.0, 20.0):
        cache = {}
        G, X, Ys, Yt = pipeline(snr, cache)
        acc = float((recognise(Ys, Yt) == lte).mean())
        snr_g = snr_of(torch, G, G64)
        holder = {}

        def step(ev, snr=snr, cache=cache, X=X, holder=holder):
            if ev is not None:
                ev[0].record(stream)
            holder["out"] = pipeline(snr, cache, X)
            if ev is not None:
                ev[1].record(stream)

        # 100 untimed pipelines (about 25 ms) so that the clocks are steady for every row
        ms, _ = timed_steps(torch, step, PCA_WARMUP, max(5, args.steps // 2), 1)
        name = "plain FP32" if snr is None else f"S = {snr:g} dB"
        rows.append({"gemms": name, "ms": round(ms, 4), "gflops": round(flops / ms / 1e6, 1),
                     "snr_G_db": round(snr_g, 2), "accuracy": round(acc, 4)})
        log(f"[bench] 2D-PCA {name:12s}: GEMMs {ms:.3f} ms -> {flops / ms / 1e6:.1f} GFLOP/s, "
            f"SNR(G) {snr_g:.2f} dB, recognition {100 * acc:.1f} %")
    main = next(r for r in rows if r["gemms"] == "S = 30 dB")
    out = {
        "metric": "effective GFLOP/s at fixed output SNR vs plain FP64 GEMM; % of FP64 MFMA peak",
        "value": main["gflops"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": max(5, args.steps // 2),
        "warmup": PCA_WARMUP,
        "ms_per_step": main["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2D-PCA on {n_tr} + {n_te} synthetic {size} x {size} images, d = {d}: the "
                               f"scatter and projection GEMMs with FP32 packing, {args.form}, L = {L}, "
                               f"S = 30 dB (also native, 40 and 20 dB and plain FP32)",
                   "parallelism": "single GPU"},
        "table": rows,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def run_scatter(args):
    """Scatter matrix X^T X and projection X P (FP32 inputs, FP64 packing)."""
    import torch

    import workloads
    from paper_1110_5765_amd import tdgemm as td

    L = args.L
    xs, ps = workloads.scatter()
    X = torch.from_numpy(xs).cuda()
    P = torch.from_numpy(ps).cuda()
    calib, _, _ = calibrate_gpu(td, torch, L, args.form, "f64", [2, 4])
    stream = torch.cuda.current_stream()
    log(f"[bench] scatter workload: X {tuple(xs.shape)} float32, P {tuple(ps.shape)}; packed FP64 "
        f"{args.form} L={L}")
    products = {"XtX": (X.t(), X), "XP": (X, P)}
    res = {}
    for name, (A, B) in products.items():
        M, K = A.shape
        N = B.shape[1]
        flops = 2.0 * M * N * K
        ref = torch.matmul(A.double(), B.double())
        res[name] = {"M": M, "N": N, "K": K}
        for S in (50.0, 40.0, 20.0):
            ks = td.auto_k_split(M, N, K, L, "f64") if args.k_split else 1
            desc = td.make_desc(A, B, L=L, form=args.form, prec="f64", ctrl="snr", snr_db=S,
                                w_allowed=(1, 2, 4), k_split=ks)
            ws = torch.empty(td.tdgemm_workspace_size(desc), dtype=torch.uint8, device="cuda")
            C = torch.empty((M, N), dtype=torch.float64, device="cuda")
            holder = {}

            def step(ev, desc=desc, ws=ws, C=C, holder=holder, A=A, B=B):
                if ev is not None:
                    ev[0].record(stream)
                holder["plan"] = td.tdgemm_plan(desc, A, B, calib, ws)
                td.tdgemm_gemm(holder["plan"], A, B, C, fused=1)
                if ev is not None:
                    ev[1].record(stream)

            ms, _ = timed_steps(torch, step, 5, max(5, args.steps // 2), 1)
            _, _, pairs, _ = td.tdgemm_plan_export(holder["plan"])
            wh = {int(w): int((pairs["w"] == w).sum()) for w in (1, 2, 4)}
            snr = snr_of(torch, C, ref)
            res[name][f"S{S:g}"] = {"ms": round(ms, 4), "gflops": round(flops / ms / 1e6, 1),
                                    "snr_db": round(snr, 2), "w_histogram": wh, "k_split": ks}
            log(f"[bench] {name} ({M}x{K} by {K}x{N}) S={S:g}: {ms:.3f} ms -> {flops / ms / 1e6:.1f} "
                f"effective GFLOP/s at {snr:.2f} dB, W {wh}")
        A64, B64 = A.double(), B.double()
        p = time_plain(torch, A64, B64, ref, reps=10)
        res[name].update(p)
        log(f"[bench] {name} plain FP64 {p['plain_fp64_gflops']} GFLOP/s, plain FP32 "
            f"{p['plain_fp32_gflops']} GFLOP/s at {p['plain_fp32_snr_db']} dB")
    main = res["XtX"]["S40"]
    out = {
        "metric": "effective GFLOP/s at fixed output SNR vs plain FP64 GEMM; % of FP64 MFMA peak",
        "value": main["gflops"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": max(5, args.steps // 2),
        "warmup": 5,
        "ms_per_step": main["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"scatter matrix X^T X, X = 2000 x 10304 mean-removed uniform float32, packed "
                               f"FP64 {args.form} L = {L}, S = 40 dB (also X P and S = 50 / 20 dB)",
                   "parallelism": "single GPU"},
        "snr_db": main["snr_db"],
        "products": res,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def precision_cpu_baseline(A, B, corner: int = 1024):
    """The oracle's INT8 form on the corner A[:c] B[:, :c] (full K), extrapolated:
    block statistics scale with the blocks of A and B, the rest with the inner kernels."""
    from threadpoolctl import threadpool_limits

    from oracle import blocks as bk
    from oracle import precision as pr

    n = A.shape[0]
    Ac, Bc = A[:corner], B[:, :corner]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        pr.run(Ac, Bc, 128, "i8", 127.0, keep_products=False)
        t1 = time.perf_counter()
        bk.all_block_stats(Ac, 128)
        bk.all_block_stats(Bc, 128)
        t2 = time.perf_counter()
    t_stats = t2 - t1
    t_rest = max((t1 - t0) - t_stats, 0.0)
    f = n / corner
    total = t_stats * f + t_rest * f * f
    model, ncpu = host_cpu()
    return {"value": 2.0 * n ** 3 / total / 1e9, "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "cpu_model": model, "nproc": ncpu,
            "sample": f"INT8 form on the {corner} x {n} by {n} x {corner} corner ({t1 - t0:.1f} s), "
                      f"statistics scaled by {f:g}, the rest by {f * f:g}"}


def host_cpu() -> tuple[str, int]:
    """(CPU model name, logical CPUs this process may run on)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


_CPU_WORKER: dict = {}


def _cpu_worker_init(dist, n, L, cfg, tabs):
    """Spawned oracle worker: one BLAS thread, its own copy of the seeded inputs."""
    from threadpoolctl import threadpool_limits

    import workloads
    _CPU_WORKER["limits"] = threadpool_limits(limits=1)
    A, B = workloads.sweep(dist, n=n)
    _CPU_WORKER.update(A=A, B=B, L=L, cfg=cfg, tabs=tabs)


def _cpu_ready(_):
    return True


def _cpu_stats_task(k):
    """Statistics of block row k of A (k < nb) or block column k - nb of B."""
    from oracle import blocks as bk
    A, B, L = _CPU_WORKER["A"], _CPU_WORKER["B"], _CPU_WORKER["L"]
    nb = bk.n_blocks(A.shape[0], L)
    if k < nb:
        return [bk.block_stats(A, k, l, L) for l in range(bk.n_blocks(A.shape[1], L))]
    return [bk.block_stats(B, l, k - nb, L) for l in range(bk.n_blocks(B.shape[0], L))]


def _cpu_tile_task(tile):
    """Plan and pipeline of one inner kernel as the sub-problem of its A row panel
    and B column panel; returns (seconds, of which the statistics of its blocks)."""
    from oracle import blocks as bk
    from oracle import pipeline as pl
    A, B, L, cfg, tabs = (_CPU_WORKER[k] for k in ("A", "B", "L", "cfg", "tabs"))
    i, j = tile
    a, b = A[i * L:(i + 1) * L], B[:, j * L:(j + 1) * L]
    t0 = time.perf_counter()
    pl.run(a, b, cfg, tabs, plan=pl.make_plan(a, b, cfg, tabs))
    t1 = time.perf_counter()
    bk.all_block_stats(a, L)
    bk.all_block_stats(b, L)
    return t1 - t0, time.perf_counter() - t1


def cpu_baseline(A, B, args):
    """The oracle on the host, on one thread and on all the cores this process may
    use. One thread: statistics of every block, then plan (options, pruning) and
    pipeline for a sample of inner kernels, extrapolated to all of them. All
    cores: spawned workers compute the statistics of all blocks (block rows of A,
    block columns of B) and the sampled inner kernels in parallel; the tile phase
    is extrapolated the same way. Its calibration table comes from the oracle's
    own measurement (untimed, like the GPU's)."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads
    from oracle import blocks as bk
    from oracle import calibration as cal
    from oracle import pipeline as pl

    L, n = args.L, A.shape[0]
    model, ncpu = host_cpu()
    workers = max(1, min(16, ncpu))
    ws_allowed = tuple(int(x) for x in args.w.split(","))
    cfg = pl.Config(L=L, form=args.form, prec="f64", ctrl="snr", snr_db=args.snr, w_allowed=ws_allowed)
    nb = bk.n_blocks(n, L)
    rng = np.random.default_rng(0)
    with threadpool_limits(limits=1):
        ua, ub = workloads.calib_uniforms(L)
        tabs = {W: cal.calibrate(L, W, args.form, "f64", ua, ub, q_max=1 << 18)[0] for W in ws_allowed if W > 1}
        tiles = [(int(i), int(j)) for i, j in rng.integers(0, nb, (args.cpu_tiles, 2))]
        t0 = time.perf_counter()
        bk.all_block_stats(A, L)
        bk.all_block_stats(B, L)
        t1 = time.perf_counter()
        plan = pl.make_plan(A, B, cfg, tabs, tiles=tiles)      # statistics again + options for the sample
        t2 = time.perf_counter()
        pl.run(A, B, cfg, tabs, tiles=tiles, plan=plan)
        t3 = time.perf_counter()
    t_stats = t1 - t0
    t_tile = max((t2 - t1) - t_stats, 0.0) + (t3 - t2)        # options, pruning and pipeline of the sample
    total1 = t_stats + t_tile * (nb * nb) / len(tiles)

    ptiles = [(int(i), int(j)) for i, j in rng.integers(0, nb, (2 * workers, 2))]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers, initializer=_cpu_worker_init, initargs=(args.dist, n, L, cfg, tabs)) as pool:
        pool.map(_cpu_ready, range(workers), chunksize=1)
        p0 = time.perf_counter()
        pool.map(_cpu_stats_task, range(2 * nb), chunksize=1)
        p1 = time.perf_counter()
        res = pool.map(_cpu_tile_task, ptiles, chunksize=1)
        p2 = time.perf_counter()
    rest = sum(t - s for t, s in res) / max(sum(t for t, _ in res), 1e-12)   # share beyond statistics
    totalp = (p1 - p0) + (p2 - p1) * rest * (nb * nb) / len(ptiles)
    flops = 2.0 * n ** 3
    return {"value": round(flops / totalp / 1e9, 4), "unit": "GFLOP/s", "cores": workers, "kind": "oracle",
            "cpu_model": model, "nproc": ncpu, "value_1thread": round(flops / total1 / 1e9, 4),
            "sample": f"1 thread: statistics of all {2 * nb * nb} blocks ({t_stats:.1f} s) plus plan and "
                      f"pipeline of {len(tiles)} of {nb * nb} inner kernels ({t_tile:.1f} s), extrapolated; "
                      f"{workers} processes: all statistics ({p1 - p0:.1f} s) plus {len(ptiles)} inner "
                      f"kernels ({p2 - p1:.1f} s, of which {100 * rest:.0f} % beyond their statistics), "
                      f"extrapolated"}


if __name__ == "__main__":
    main()
