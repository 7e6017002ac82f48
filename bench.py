"""Throughput of the RK4IP step on one MI355X, with roofline and CPU baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload wdm36]
                    [--precision fp32|split_bf16|split_bf16_s] [--no-cpu-baseline]

A step is one RK4IP step (Eq. 6a-f of the paper: four half-step propagators,
four Kerr evaluations, the stage combinations) over the whole field.  The
field and all tables are resident in HBM before the timed region; the timed
region is K calls' worth of device work launched by mmnlse_advance,
bracketed by synchronisation.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RK4IP mode·sample·steps/s + roofline %, plain vs split-BF16; p50/p99 latency"
PRECISIONS = ("fp32", "split_bf16", "split_bf16_s")
DTYPES = {"fp32": "f32", "split_bf16": "bf16x3-split/f32-acc", "split_bf16_s": "bf16x2-split-S/f32-acc"}


def precision_code(mm, name: str) -> int:
    return {"fp32": mm.FP32, "split_bf16": mm.SPLIT_BF16, "split_bf16_s": mm.SPLIT_BF16_S}[name]
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0

WORKLOADS = {
    "wdm36": "wdm36: M=36 modes, T=2^16 complex64, 8-ch WDM 16-QAM 32 GBd, masked symmetric S, h=50 m",
    "qpsk6": "qpsk6: M=6 modes, T=2^14 complex64, QPSK 32 GBd, dense symmetric S, h=100 m",
    "soliton": "soliton: M=1, T=4096, fundamental sech soliton, h=5 m",
    "wdm120": "wdm120: M=120 modes, T=2^17 complex64, 4-ch WDM QPSK, dense symmetric S, h=20 m",
    "manakov": "manakov: M=30 rows (15 spatial modes x 2 polarizations), T=2^16 complex64, "
               "8-ch WDM 16-QAM, Manakov/XPM operator of Eq. (1), alpha 0.23 dB/km, h=100 m",
}
METHODS = {"rk4ip": 0, "ssfm_rk4": 1, "ssfm_agrawal": 2}


def manakov_flops_per_eval(M: int, T: int) -> float:
    """Flops of one Manakov/XPM evaluation h N(X)_a = i gamma h (sum_b kappa_ab |X_b|^2) X_a:
    |X_b|^2 (3 per mode and sample), the kappa row sums (2 M^2 per sample), and
    the scaled rotation of X_a (3 per mode and sample)."""
    return (2.0 * M * M + 6.0 * M) * T


def kerr_flops_per_eval(M: int, T: int, entries: float | None = None) -> float:
    """Flops of one Kerr evaluation h N(X) in the packed form: B_q = X_l X_m
    (6 flops per pair and sample), C = S_pack B (4 flops per packed tensor
    entry and sample: a real multiply-add on Re B and on Im B), out_p =
    sum_n C_pn conj(X_n) (8 per (p,n) term, M^2 terms per sample).
    ``entries`` = packed tensor entries counted (default: all P^2; the
    algorithmic count takes only the nonzero ones)."""
    P = M * (M + 1) // 2
    if entries is None:
        entries = float(P * P)
    return 4.0 * entries * T + 6.0 * P * T + 8.0 * M * M * T


def linear_bytes_per_apply(M: int, T: int, four_step: bool) -> float:
    """Algorithmic HBM bytes of one half-step propagator application on one
    field: read + write of M*T complex64 plus the M*T hi+lo factor table
    (16 B per entry).  A four-step transform needs two more read + write
    passes (the strided column passes)."""
    passes = 3 if four_step else 1
    return M * T * (16.0 * passes + 16.0)


def cpu_baseline(p, seconds_target: float = 15.0, method: str = "rk4ip"):
    """Time the FP64 oracle on this host over a bounded number of steps."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    if getattr(p, "kappa", None) is not None:
        kern = oracle.KerrManakov(p.kappa.astype(np.float64), p.gamma)
    else:
        kern = oracle.KerrGeneric(p.S, p.gamma)
    step = {"rk4ip": oracle.rk4ip_step, "ssfm_rk4": oracle.ssfm_rk4_step,
            "ssfm_agrawal": oracle.ssfm_agrawal_step}[method]
    alpha = p.alpha if np.any(p.alpha) else None
    E = oracle.half_step_propagator(oracle.angular_frequencies(p.T, p.dt), p.beta, alpha, p.h)
    A = p.A0.astype(np.complex128)
    steps = 0
    t0 = time.perf_counter()
    while True:
        A = step(A, E, p.h, kern)
        steps += 1
        el = time.perf_counter() - t0
        if el > seconds_target or steps >= p.n_steps:
            break
    v = p.M * p.T * steps / el
    return {"value": v, "unit": "mode*sample*steps/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{steps} {method} steps of the full {p.name} field (M={p.M}, T={p.T}), FP64 numpy, "
                      f"{el:.1f} s"}


def serving(args):
    """Continuous-batching serving run: seeded Poisson request stream (M in {1,6,15,36},
    T in {2^12,2^14,2^16}, L in {1,10,50} km) submitted at its arrival times."""
    import threading

    import paper_1901_01895_amd as mm
    import workloads as W

    specs = W.serving_stream(args.requests, rate=args.rate)
    probs = [W.fiber.request_problem(sp) for sp in specs]
    prec = precision_code(mm, args.precision)
    cfgs = [mm.problem_config(p, precision=prec if p.M > 8 else mm.FP32) for p in probs]
    work = sum(p.M * p.T * p.n_steps for p in probs)
    lat = [None] * len(probs)
    with mm.Server(steps_per_tick=args.steps_per_tick, n_streams=args.streams) as srv:
        tickets = [None] * len(probs)
        t0 = time.perf_counter()

        def feeder():
            for i, (sp, p) in enumerate(zip(specs, probs)):
                dt = sp.arrival - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                tickets[i] = srv.submit(p.A0, cfgs[i])

        th = threading.Thread(target=feeder)
        th.start()
        th.join()
        for i, t in enumerate(tickets):
            _, info = srv.wait(t)
            lat[i] = info["latency"]
        el = time.perf_counter() - t0
        counters = srv.counters()
    lat = np.array(lat)
    return {
        "metric": METRIC, "value": work / el, "unit": "mode*sample*steps/s", "n_gpus": 1,
        "steps": int(sum(p.n_steps for p in probs)), "warmup": 0, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES[args.precision], "data": "synthetic",
        "config": {"workload": f"serving: {len(probs)} requests, Poisson rate "
                               f"{'saturated' if args.rate is None else args.rate}/s, M in {{1,6,15,36}}, "
                               "T in {2^12,2^14,2^16}, L in {1,10,50} km",
                   "precision": args.precision, "steps_per_tick": args.steps_per_tick,
                   "streams": args.streams},
        "latency_s": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                      "max": float(lat.max())},
        "wall_s": el, "server": counters,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="wdm36", choices=sorted(WORKLOADS) + ["serving"])
    ap.add_argument("--precision", default="fp32", choices=list(PRECISIONS),
                    help="precision of the headline value; the others are reported beside it")
    ap.add_argument("--precision-only", action="store_true", help="measure only --precision")
    ap.add_argument("--method", default="rk4ip", choices=sorted(METHODS),
                    help="step scheme (ssfm_agrawal needs the manakov workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--requests", type=int, default=256, help="serving: number of requests")
    ap.add_argument("--rate", type=float, default=None, help="serving: Poisson rate 1/s (default saturated)")
    ap.add_argument("--steps-per-tick", type=int, default=8)
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU work: write the HBM-traffic record of two rocprofv3 --pmc runs")
    args = ap.parse_args()
    if args.summarize_pmc:
        print(json.dumps(summarize_pmc(*args.summarize_pmc, args.workload, args.precision)))
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the RK4IP path here is single-device (fields and the "
              "coupling tensor fit one MI355X); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1901_01895_amd as mm
    import workloads as W

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    mm.load()
    if args.workload == "serving":
        print(json.dumps(serving(args)), flush=True)
        return
    p = W.make_problem(args.workload)
    precs = [args.precision] if args.precision_only else \
        [args.precision] + [q for q in PRECISIONS if q != args.precision]
    runs = {}
    for q in precs:
        if q != "fp32" and not p.symmetric:
            continue
        runs[q] = measure(mm, W, p, q, args)
    main_run = runs[args.precision]
    out = {
        "metric": METRIC, "value": main_run["value"], "unit": "mode*sample*steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES[args.precision], "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "M": p.M, "T": p.T, "h_km": p.h,
                   "precision": args.precision, "method": args.method,
                   "kerr_kernel": main_run["kerr_kernel"]},
        "roofline": main_run["roofline"],
        "kernels": main_run["kernels"],
    }
    for q, r in runs.items():
        if q != args.precision:
            out[q] = {k: r[k] for k in ("value", "ms_per_step", "roofline", "kernels")}
            out[q]["speedup_vs_" + args.precision] = r["value"] / main_run["value"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds, args.method)
    print(json.dumps(out), flush=True)


def summarize_pmc(fetch_dir: str, write_dir: str, workload: str, precision: str) -> dict:
    """Turn two rocprofv3 --pmc runs of this script (FETCH_SIZE, then
    WRITE_SIZE, ``--precision-only``) into profiles/<kernel>_<workload>_pmc.json.

    The counters read KiB per dispatch.  Each is scaled by what it reads for
    the plain device-to-device copy of the field that the timed region starts
    with (M*T*8 bytes read and written; the copyBuffer dispatch with the
    largest reading), and averaged over the dispatches of the dominant Kerr
    kernel, like the per-launch duration in the roofline.
    """
    import csv
    import glob
    import hashlib
    import re
    import workloads as W

    def load(d, counter):
        out = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r.get("Counter_Name") == counter:
                    key = (int(r["Dispatch_Id"]), r["Kernel_Name"])
                    out[key] = out.get(key, 0.0) + float(r["Counter_Value"])
        return out

    p = W.make_problem(workload)
    copy_bytes = float(p.M * p.T * 8)
    mode = {"fp32": "0", "split_bf16": "1", "split_bf16_s": "2"}[precision]
    pat = re.compile(r"kerr_mfma<\d+, \d+, " + mode + ",")
    fe, wr = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    rec = {"kernel": f"kerr_mfma_{precision}", "workload": workload, "source": "kerr_mfma.hip"}
    src = os.path.join(ROOT, "paper_1901_01895_amd", "csrc", rec["source"])
    rec["source_sha256"] = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for name, m in (("fetch", fe), ("write", wr)):
        copy = max([v for (_, k), v in m.items() if "copyBuffer" in k] or [0.0])
        vals = [v for (_, k), v in m.items() if pat.search(k)]
        if not copy or not vals:
            raise SystemExit(f"no {name} counters for the copy or the Kerr kernel under the given folder")
        rec[f"{name}_kib_per_launch"] = sum(vals) / len(vals)
        rec[f"{name}_launches"] = len(vals)
        rec[f"{name}_copy_kib"] = copy
        rec[f"{name}_factor"] = copy_bytes / (copy * 1024.0)
    rec["copy_bytes"] = copy_bytes
    rec["bytes_per_launch"] = 1024.0 * (rec["fetch_kib_per_launch"] * rec["fetch_factor"]
                                        + rec["write_kib_per_launch"] * rec["write_factor"])
    path = os.path.join(ROOT, "profiles", f"{rec['kernel']}_{workload}_pmc.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


def traffic_for(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it was
    taken on the current kernel source (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_1901_01895_amd", "csrc", rec["source"])
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
        return None
    return rec["bytes_per_launch"]


def measure(mm, W, p, precision: str, args) -> dict:
    import torch
    prec = precision_code(mm, precision)
    P = mm.Propagator.from_problem(p, precision=prec, method=METHODS[args.method])
    A0 = torch.from_numpy(p.A0.astype(np.complex64)).cuda()
    A = A0.clone()

    # warmup
    P.advance(A, args.warmup)
    torch.cuda.synchronize()
    # timed region
    A.copy_(A0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.advance(A, args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_per_step = 1e3 * el / args.steps
    value = p.M * p.T * args.steps / el

    # per-kernel device time (HIP events on the plan's stream), same step count
    B = A0.clone()
    prof = P.profile(B, args.steps)
    four = p.T > 16384
    kerr_avg_ms = prof["kerr_ms"] / max(prof["kerr_launches"], 1)
    lin_avg_ms = prof["linear_ms"] / max(prof["linear_launches"], 1)
    path = P.kerr_path
    work = P.kerr_work() if path == "mfma" else None
    # algorithmic: nonzero tensor entries only; executed: the blocks the kernel multiplies
    if path == "manakov":
        kflops = xflops = manakov_flops_per_eval(p.M, p.T)
    else:
        kflops = kerr_flops_per_eval(p.M, p.T, work["nonzero"] if work else None)
        xflops = kerr_flops_per_eval(p.M, p.T, work["multiplied"] if work else None)
    evals_per_launch = prof["kerr_evals"] / max(prof["kerr_launches"], 1)
    kerr_tflops = kflops * evals_per_launch / (kerr_avg_ms * 1e-3) / 1e12
    exec_tflops = xflops * evals_per_launch / (kerr_avg_ms * 1e-3) / 1e12
    # RK4IP's linear launches carry two fields (A and k1, then the two stage sums);
    # the split-step schemes transform one field per launch
    fields = 2 if args.method == "rk4ip" else 1
    lin_gbs = fields * linear_bytes_per_apply(p.M, p.T, four) / (lin_avg_ms * 1e-3) / 1e9
    kerr_dominant = prof["kerr_ms"] >= prof["linear_ms"]
    if kerr_dominant and path == "manakov":
        # pointwise in t with O(M) work per sample: bound by the field passes
        # (per step RK4IP's fused K2+K3 and K4 launches read + write 4 fields
        # each, SSFM-RK4 adds the plain k1 launch (2) and its K4 writes one
        # field (3), the Agrawal phase launches read 3 and write 1)
        passes = {"rk4ip": 8, "ssfm_rk4": 9, "ssfm_agrawal": 8}[args.method]
        kname = f"kerr_manakov_{precision}"
        kgbs = passes * p.M * p.T * 8.0 / (prof["kerr_ms"] / args.steps * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": kgbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": kgbs / HBM_PEAK_GBS, "traffic": None, "kernel": kname,
                "avg_launch_ms": kerr_avg_ms, "field_passes_per_step": passes}
    elif kerr_dominant:
        if path == "mfma" and prec != mm.FP32:
            bound, peak = "mfma", BF16_PEAK_TFLOPS
        elif path == "mfma":
            bound, peak = "mfma", FP32_PEAK_TFLOPS
        else:
            bound, peak = "alu", FP32_PEAK_TFLOPS
        kname = f"kerr_{path}_{precision}"
        roof = {"bound": bound, "achieved": kerr_tflops, "peak": peak, "unit": "TFLOP/s",
                "frac": kerr_tflops / peak, "traffic": traffic_for(kname, args.workload),
                "kernel": kname, "avg_launch_ms": kerr_avg_ms,
                "evals_per_launch": evals_per_launch,
                "flops_per_eval": kflops, "executed_tflops": exec_tflops,
                "nonzero_fraction": work["nonzero"] / work["dense"] if work else 1.0,
                "multiplied_fraction": work["multiplied"] / work["dense"] if work else 1.0}
    else:
        kname = "linear_half_step"
        roof = {"bound": "hbm", "achieved": lin_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": lin_gbs / HBM_PEAK_GBS, "traffic": traffic_for(kname, args.workload),
                "kernel": kname, "avg_launch_ms": lin_avg_ms}
    P.close()
    return {"value": value, "ms_per_step": ms_per_step, "roofline": roof, "kerr_kernel": path,
            "kernels": {"kerr_ms_per_step": prof["kerr_ms"] / args.steps, "kerr_executed_tflops": exec_tflops,
                        "linear_ms_per_step": prof["linear_ms"] / args.steps,
                        "kerr_tflops": kerr_tflops, "linear_GBps": lin_gbs}}


if __name__ == "__main__":
    main()
