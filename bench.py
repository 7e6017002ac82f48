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
FULL_T = {"wdm36": 2 ** 16, "qpsk6": 2 ** 14, "soliton": 4096, "wdm120": 2 ** 17, "manakov": 2 ** 16}


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


def linear_bytes_per_apply(M: int, T: int) -> float:
    """Algorithmic HBM bytes of one half-step propagator application on one
    field: read + write of M*T complex64 plus the M*T hi+lo factor table
    (16 B per entry), 32 B per sample.  (A four-step transform moves the field
    through HBM three times, 64 B per sample; that is executed traffic, not
    the algorithm's.)"""
    return M * T * 32.0


def cpu_model() -> str:
    """CPU model name of this host (from /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _time_oracle(p, kern, step, E, alpha, seconds_target: float):
    A = p.A0.astype(np.complex128)
    steps = 0
    t0 = time.perf_counter()
    while True:
        A = step(A, E, p.h, kern)
        steps += 1
        el = time.perf_counter() - t0
        if el > seconds_target or steps >= p.n_steps:
            break
    return steps, el


def cpu_baseline(p, seconds_target: float = 15.0, method: str = "rk4ip"):
    """Time the FP64 oracle on this host over a bounded number of steps, with
    numpy's BLAS on every core it may use and again on one thread."""
    import oracle
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    if getattr(p, "kappa", None) is not None:
        kern = oracle.KerrManakov(p.kappa.astype(np.float64), p.gamma)
    else:
        kern = oracle.KerrGeneric(p.S, p.gamma)
    step = {"rk4ip": oracle.rk4ip_step, "ssfm_rk4": oracle.ssfm_rk4_step,
            "ssfm_agrawal": oracle.ssfm_agrawal_step}[method]
    alpha = p.alpha if np.any(p.alpha) else None
    E = oracle.half_step_propagator(oracle.angular_frequencies(p.T, p.dt), p.beta, alpha, p.h)
    steps, el = _time_oracle(p, kern, step, E, alpha, seconds_target)
    with threadpool_limits(limits=1):
        steps1, el1 = _time_oracle(p, kern, step, E, alpha, seconds_target / 2)
    v = p.M * p.T * steps / el
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        affinity = os.cpu_count() or 1
    return {"value": v, "unit": "mode*sample*steps/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{steps} {method} steps of the full {p.name} field (M={p.M}, T={p.T}), FP64 numpy, "
                      f"{el:.1f} s",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "affinity_cpus": affinity,
            "blas_threads": int(threads),
            "one_thread": {"value": p.M * p.T * steps1 / el1, "steps": steps1, "seconds": el1}}


def serving(args, precision: str | None = None, rate: float | None = None, n_requests: int | None = None):
    """Continuous-batching serving run: seeded Poisson request stream (M in {1,6,15,36},
    T in {2^12,2^14,2^16}, L in {1,10,50} km) submitted at its arrival times.
    ``precision``, ``rate`` and ``n_requests`` default to the command line's."""
    import threading

    import paper_1901_01895_amd as mm
    import workloads as W

    precision = precision or args.precision
    rate = args.rate if rate is None and args.workload == "serving" else rate
    specs = W.serving_stream(n_requests or args.requests, rate=rate)
    probs = [W.fiber.request_problem(sp) for sp in specs]
    prec = precision_code(mm, precision)
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
        "dtype": DTYPES[precision], "data": "synthetic",
        "config": {"workload": f"serving: {len(probs)} requests, Poisson rate "
                               f"{'saturated' if rate is None else rate}/s, M in {{1,6,15,36}}, "
                               "T in {2^12,2^14,2^16}, L in {1,10,50} km",
                   "precision": precision, "steps_per_tick": args.steps_per_tick,
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
    ap.add_argument("--no-serving", action="store_true",
                    help="leave out the serving runs of the default report")
    ap.add_argument("--serving-rate", type=float, default=3.6,
                    help="Poisson rate 1/s of the default report's latency runs")
    ap.add_argument("--serving-requests", type=int, default=128,
                    help="requests per run of the default report's serving runs")
    ap.add_argument("--full-length", action="store_true",
                    help="run the workload's whole length (L/h steps) in FP32 and split-bf16 and report the FP64 "
                         "power drift and the split-vs-FP32 difference (no throughput line)")
    ap.add_argument("--summarize-stats", metavar="DIR",
                    help="no GPU work: write the kernel-statistics record of a rocprofv3 --stats run")
    ap.add_argument("--summarize-sq", nargs="+", metavar="DIR",
                    help="no GPU work: write the SQ counter record of rocprofv3 --pmc runs")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU work: write the HBM-traffic record of two rocprofv3 --pmc runs")
    args = ap.parse_args()
    if args.summarize_pmc:
        print(json.dumps(summarize_pmc(*args.summarize_pmc, args.workload, args.precision)))
        return
    if args.summarize_stats:
        rec = summarize_stats(args.summarize_stats, args.workload, args.precision, args.steps, args.warmup)
        print(json.dumps({k: v for k, v in rec.items() if k != "kernels"}))
        return
    if args.summarize_sq:
        print(json.dumps(summarize_sq(args.summarize_sq, args.workload, args.precision)["ratios"]))
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
    if args.full_length:
        print(json.dumps(full_length(mm, W, p, args)), flush=True)
        return
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
    if not args.no_serving and args.workload == "wdm36" and args.method == "rk4ip":
        out["serving"] = serving_report(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds, args.method)
    print(json.dumps(out), flush=True)


def full_length(mm, W, p, args) -> dict:
    """The whole propagation (L/h RK4IP steps) of the workload in FP32, split
    bf16 (three products) and split-S: FP64 power in and out (conserved for
    alpha = 0 and a symmetric tensor), wall time, and the relative L2
    difference of each split result from the FP32 one.  Progress to stderr."""
    import torch
    A0 = torch.from_numpy(p.A0.astype(np.complex64)).cuda()
    res, fields = {}, {}
    chunk = max(1, p.n_steps // 10)
    for q in ("fp32", "split_bf16", "split_bf16_s"):
        P = mm.Propagator.from_problem(p, precision=precision_code(mm, q))
        A = A0.clone()
        pin = P.power(A)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < p.n_steps:
            n = min(chunk, p.n_steps - done)
            P.advance(A, n)
            torch.cuda.synchronize()
            done += n
            print(f"bench: full length {p.name} {q}: step {done}/{p.n_steps} ({time.perf_counter() - t0:.0f} s)",
                  file=sys.stderr, flush=True)
        el = time.perf_counter() - t0
        pout = P.power(A)
        P.close()
        fields[q] = A.cpu().numpy()
        res[q] = {"steps": p.n_steps, "seconds": el, "ms_per_step": 1e3 * el / p.n_steps,
                  "power_in_W_ps": pin, "power_out_W_ps": pout, "power_drift": pout / pin - 1.0}
    ref = fields["fp32"].astype(np.complex128)
    nref = np.linalg.norm(ref)
    for q in ("split_bf16", "split_bf16_s"):
        d = fields[q].astype(np.complex128) - ref
        res[q]["rel_l2_vs_fp32"] = float(np.linalg.norm(d) / nref)
        res[q]["worst_mode_rel_l2_vs_fp32"] = float(np.max(np.linalg.norm(d, axis=1) / np.linalg.norm(ref, axis=1)))
    return {"workload": WORKLOADS.get(args.workload, args.workload), "M": p.M, "T": p.T, "h_km": p.h,
            "L_km": p.h * p.n_steps, "results": res}


def serving_report(args) -> dict:
    """The serving part of the metric beside the throughput line: the seeded
    stream of --serving-requests requests saturated (every arrival at t = 0:
    throughput) and as a Poisson stream at --serving-rate (p50/p99 latency),
    each with the plain FP32 and the split-bf16 contraction.  Progress goes to
    stderr."""
    runs = []
    for rate in (None, args.serving_rate):
        for q in ("fp32", "split_bf16"):
            r = serving(args, precision=q, rate=rate, n_requests=args.serving_requests)
            runs.append({"arrivals": "saturated" if rate is None else f"poisson {rate}/s", "precision": q,
                         "value": r["value"], "unit": r["unit"], "latency_s": r["latency_s"],
                         "wall_s": r["wall_s"], "ticks": r["server"]["rounds"]})
            print(f"bench: serving {runs[-1]['arrivals']} {q}: {r['value']:.3e} {r['unit']}, "
                  f"p50 {r['latency_s']['p50']:.3f} s, p99 {r['latency_s']['p99']:.3f} s", file=sys.stderr, flush=True)
    head = next(r for r in runs if r["arrivals"] != "saturated" and r["precision"] == args.precision
                ) if args.precision in ("fp32", "split_bf16") else runs[-1]
    sat = next(r for r in runs if r["arrivals"] == "saturated" and r["precision"] == head["precision"])
    return {"requests": args.serving_requests, "precision": head["precision"], "latency_s": head["latency_s"],
            "poisson_rate_per_s": args.serving_rate, "saturated_value": sat["value"], "unit": sat["unit"],
            "runs": runs}


def summarize_pmc(fetch_dir: str, write_dir: str, workload: str, precision: str) -> dict:
    """Turn two rocprofv3 --pmc runs of
        bench.py --workload <w> --steps K --warmup W --no-cpu-baseline --no-serving
    (FETCH_SIZE, then WRITE_SIZE) into profiles/kerr_<p>_<w>_pmc.json for
    precision p: HBM bytes per launch of p's Kerr kernels.

    The counters read KiB per dispatch.  Each is scaled by what it reads for
    the plain device-to-device copy of the field that the timed region starts
    with (M*T*8 bytes read and written; the copyBuffer dispatch with the
    largest reading), and averaged over the dispatches of p's Kerr kernels,
    like the per-launch duration in the roofline.
    """
    import csv
    import glob
    import workloads as W

    def load(d, counter):
        out = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r.get("Counter_Name") == counter:
                    key = (int(r["Dispatch_Id"]), r["Kernel_Name"])
                    out[key] = out.get(key, 0.0) + float(r["Counter_Value"])
        return out

    p = W.make_problem(workload, T=256, n_steps=1)
    copy_bytes = float(p.M * FULL_T[workload] * 8)
    fe, wr = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    rec = {"workload": workload, "precision": precision, "csrc_sha256": csrc_digest(),
           "command": (f"cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) "
                       f"--output-format csv -d <dir> -o run -- python3 <repo>/bench.py --workload {workload} "
                       f"--steps <K> --warmup <W> --no-cpu-baseline --no-serving; python3 bench.py "
                       f"--summarize-pmc <fetch dir> <write dir> --workload {workload} --precision {precision}")}
    for name, m in (("fetch", fe), ("write", wr)):
        copy = max([v for (_, k), v in m.items() if "copyBuffer" in k] or [0.0])
        vals = [v for (_, k), v in m.items() if kerr_kernel_precision(k) == precision]
        if not copy or not vals:
            raise SystemExit(f"no {name} counters for the copy or the {precision} Kerr kernels under the given folder")
        rec[f"{name}_kib_per_launch"] = sum(vals) / len(vals)
        rec[f"{name}_launches"] = len(vals)
        rec[f"{name}_copy_kib"] = copy
        rec[f"{name}_factor"] = copy_bytes / (copy * 1024.0)
    rec["copy_bytes"] = copy_bytes
    rec["bytes_per_launch"] = 1024.0 * (rec["fetch_kib_per_launch"] * rec["fetch_factor"]
                                        + rec["write_kib_per_launch"] * rec["write_factor"])
    path = os.path.join(ROOT, "profiles", f"kerr_{precision}_{workload}_pmc.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


def csrc_digest() -> str:
    """sha256 over the library's HIP sources (names and contents, sorted)."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1901_01895_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def _kerr_flops(workload: str, precision: str) -> tuple[float, float]:
    """(algorithmic flops per Kerr evaluation, flops of the blocks the plan
    multiplies) for a workload, from the host-only contraction plan."""
    import paper_1901_01895_amd as mm
    import workloads as W
    p = W.make_problem(workload, T=256, n_steps=1)  # same tensor as the full field
    plan = mm.kerr_plan(p.S, precision_code(mm, precision))
    T = FULL_T[workload]
    e = plan["entries"]
    return kerr_flops_per_eval(p.M, T, e["nonzero"]), kerr_flops_per_eval(p.M, T, e["multiplied"])


def kerr_kernel_precision(name: str):
    """Precision of a matrix-core Kerr kernel from its template arguments
    (kerr_mfma<W, R, SPLIT, ...>, kerr_group<TT, RW, NPART, KC, SPLIT, ...>), else None."""
    import re
    m = re.search(r"kerr_(mfma|group)<([^>]*)>", name)
    if not m:
        return None
    args = [a.strip() for a in m.group(2).split(",")]
    split = args[2] if m.group(1) == "mfma" else args[4]
    return {"0": "fp32", "1": "split_bf16", "2": "split_bf16_s"}.get(split)


def summarize_stats(stats_dir: str, workload: str, precision: str, steps: int, warmup: int) -> dict:
    """Turn a rocprofv3 --kernel-trace --stats run of
        bench.py --workload <w> --steps K --warmup W --no-cpu-baseline --no-serving
    (every precision measured in one process, as in the default report) into
    profiles/kerr_<p>_<w>_stats.json for precision p: the calls and average
    duration of every kernel of the run, and the Kerr time per evaluation on
    the basis of the bench line's roofline (the durations of p's Kerr kernels
    over the 4 evaluations of every RK4IP step measure() made for p: W warmup,
    K timed, K profiled)."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(stats_dir, "**", "*kernel_stats.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            rows.append({"name": r["Name"], "calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"]),
                         "total_ns": float(r["TotalDurationNs"])})
    if not rows:
        raise SystemExit("no kernel_stats.csv under " + stats_dir)
    kerr = [r for r in rows if kerr_kernel_precision(r["name"]) == precision]
    lin = [r for r in rows if "linear_" in r["name"]]
    if not kerr:
        raise SystemExit(f"no {precision} Kerr kernels in {stats_dir}")
    total_steps = warmup + 2 * steps
    evals = 4 * total_steps
    kerr_ms = sum(r["total_ns"] for r in kerr) * 1e-6
    flops, xflops = _kerr_flops(workload, precision)
    ms_eval = kerr_ms / evals
    peak = FP32_PEAK_TFLOPS if precision == "fp32" else BF16_PEAK_TFLOPS
    rec = {"workload": workload, "precision": precision, "csrc_sha256": csrc_digest(),
           "command": (f"cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats --output-format csv "
                       f"-d <dir> -o run -- python3 <repo>/bench.py --workload {workload} "
                       f"--steps {steps} --warmup {warmup} --no-cpu-baseline --no-serving; "
                       f"python3 bench.py --summarize-stats <dir> --workload {workload} --precision {precision} "
                       f"--steps {steps} --warmup {warmup}"),
           "rk4ip_steps": total_steps, "kerr_evals": evals,
           "kerr_ms_per_step": kerr_ms / total_steps, "kerr_ms_per_eval": ms_eval,
           # the linear kernels serve every precision the run measured
           "linear_ms_per_step": sum(r["total_ns"] for r in lin) * 1e-6 / (total_steps * max(1, len(
               {kerr_kernel_precision(r["name"]) for r in rows} - {None}))),
           "flops_per_eval": flops, "executed_flops_per_eval": xflops,
           "achieved_tflops": flops / (ms_eval * 1e-3) / 1e12,
           "executed_tflops": xflops / (ms_eval * 1e-3) / 1e12,
           "peak_tflops": peak, "frac": flops / (ms_eval * 1e-3) / 1e12 / peak,
           "kernels": sorted(rows, key=lambda r: -r["total_ns"])}
    path = os.path.join(ROOT, "profiles", f"kerr_{precision}_{workload}_stats.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


def summarize_sq(dirs: list[str], workload: str, precision: str) -> dict:
    """SQ / GRBM counters of precision p's Kerr kernels from rocprofv3 --pmc
    runs of bench.py --workload <w> --no-cpu-baseline --no-serving (one counter
    set per run) into profiles/kerr_<p>_<w>_sq.json, with
    per-wave ratios and the matrix-core busy fraction
        SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 XCDs * 256 CUs * 4 SIMDs)."""
    import csv
    import glob
    tot: dict = {}
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if kerr_kernel_precision(r["Kernel_Name"]) == precision:
                    tot[r["Counter_Name"]] = tot.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    if not tot:
        raise SystemExit("no Kerr kernel counters under the given folders")
    rec = {"workload": workload, "precision": precision, "csrc_sha256": csrc_digest(),
           "command": ("cd /tmp && export TMPDIR=/tmp && rocprofv3 --pmc <counter set> --output-format csv -d <dir> "
                       f"-o run -- python3 <repo>/bench.py --workload {workload} --steps <K> --warmup <W> "
                       f"--no-cpu-baseline --no-serving (one run per set); python3 bench.py --summarize-sq <dirs> "
                       f"--workload {workload} --precision {precision}"),
           "counters": tot}
    wc = tot.get("SQ_WAVE_CYCLES")
    ratios = {}
    for k in ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_WAIT_INST_LDS", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS",
              "SQ_ACTIVE_INST_ANY", "SQ_ACTIVE_INST_VMEM"):
        if wc and k in tot:
            ratios[k + "/SQ_WAVE_CYCLES"] = tot[k] / wc
    if tot.get("SQ_INSTS_MFMA"):
        ratios["SQ_INSTS_VALU/SQ_INSTS_MFMA"] = tot.get("SQ_INSTS_VALU", 0.0) / tot["SQ_INSTS_MFMA"]
        ratios["SQ_INSTS_LDS/SQ_INSTS_MFMA"] = tot.get("SQ_INSTS_LDS", 0.0) / tot["SQ_INSTS_MFMA"]
    if tot.get("GRBM_GUI_ACTIVE") and "SQ_VALU_MFMA_BUSY_CYCLES" in tot:
        ratios["mfma_busy"] = tot["SQ_VALU_MFMA_BUSY_CYCLES"] / (tot["GRBM_GUI_ACTIVE"] / 8 * 256 * 4)
    rec["ratios"] = ratios
    path = os.path.join(ROOT, "profiles", f"kerr_{precision}_{workload}_sq.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


def rocprof_record(workload: str, precision: str):
    """The committed kernel-statistics summary for this workload and precision,
    if it was taken on the current sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"kerr_{precision}_{workload}_stats.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    return rec if rec.get("csrc_sha256") == csrc_digest() else None


def traffic_for(precision: str, workload: str):
    """HBM bytes per launch of the Kerr kernels from the committed rocprofv3
    counter record, if it was taken on the current sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"kerr_{precision}_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    return rec["bytes_per_launch"] if rec.get("csrc_sha256") == csrc_digest() else None


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
    four = p.T > 16384 or (p.T >= 4096 and 2 * p.M < 128)  # the plan's choice of the four-step transform
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
    # (plans that run whole steps in one workgroup make no separate linear launches)
    lin_gbs = fields * linear_bytes_per_apply(p.M, p.T) / (lin_avg_ms * 1e-3) / 1e9 if lin_avg_ms > 0 else 0.0
    lin_exec_gbs = lin_gbs * (2.0 if four else 1.0)
    kerr_dominant = prof["kerr_ms"] >= prof["linear_ms"]
    solo = prof["linear_launches"] == 0 and args.method == "rk4ip" and p.M == 1
    if solo:
        # one mode: whole steps in one workgroup (one launch per call), bound by
        # one CU's FP32 rate; algorithmic flops per step = 8 transforms of
        # 5 T log2 T, 4 propagator products and 4 Kerr evaluations of 6 T each
        sflops = 8 * 5.0 * p.T * math.log2(p.T) + 4 * 2 * 6.0 * p.T + 4 * 8.0 * p.T
        cu_peak = FP32_PEAK_TFLOPS / 256
        stf = sflops / (prof["kerr_ms"] / args.steps * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": stf, "peak": cu_peak, "unit": "TFLOP/s", "frac": stf / cu_peak,
                "traffic": None, "kernel": "rk4ip_solo", "peak_basis": "one CU (one workgroup)",
                "avg_launch_ms": kerr_avg_ms, "flops_per_step": sflops}
    elif kerr_dominant and path == "manakov":
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
                "frac": kerr_tflops / peak, "traffic": traffic_for(precision, args.workload),
                "kernel": kname, "avg_launch_ms": kerr_avg_ms,
                "evals_per_launch": evals_per_launch,
                "flops_per_eval": kflops, "executed_tflops": exec_tflops,
                "nonzero_fraction": work["nonzero"] / work["dense"] if work else 1.0,
                "multiplied_fraction": work["multiplied"] / work["dense"] if work else 1.0,
                "kerr_ms_per_eval": prof["kerr_ms"] / max(prof["kerr_evals"], 1)}
        rec = rocprof_record(args.workload, precision) if args.method == "rk4ip" else None
        if rec is not None:
            # the committed rocprofv3 kernel statistics of the same sources, on
            # the same basis (Kerr kernel time per evaluation)
            roof["rocprof"] = {"kerr_ms_per_eval": rec["kerr_ms_per_eval"], "frac": rec["frac"],
                               "events_over_rocprof": roof["kerr_ms_per_eval"] / rec["kerr_ms_per_eval"],
                               "record": f"profiles/kerr_{precision}_{args.workload}_stats.json"}
    else:
        kname = "linear_half_step"
        roof = {"bound": "hbm", "achieved": lin_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": lin_gbs / HBM_PEAK_GBS, "traffic": None,
                "kernel": kname, "avg_launch_ms": lin_avg_ms, "executed_GBps": lin_exec_gbs}
    P.close()
    return {"value": value, "ms_per_step": ms_per_step, "roofline": roof, "kerr_kernel": path,
            "kernels": {"kerr_ms_per_step": prof["kerr_ms"] / args.steps, "kerr_executed_tflops": exec_tflops,
                        "linear_ms_per_step": prof["linear_ms"] / args.steps,
                        "kerr_tflops": kerr_tflops, "linear_GBps": lin_gbs, "linear_executed_GBps": lin_exec_gbs}}


if __name__ == "__main__":
    main()
