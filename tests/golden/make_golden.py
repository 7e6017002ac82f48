"""Write stored FP64-oracle samples for the long parity checks.

    python tests/golden/make_golden.py wdm36 --checkpoints 10 100 300 1000
    python tests/golden/make_golden.py wdm120 --checkpoints 1 5

Calls only ``oracle/`` on inputs from ``workloads/`` (nothing from the GPU
library).  wdm36 runs the generic Kerr form (no symmetry assumed, the plain
definition); wdm120 the packed form over the pairs l <= m, which the oracle
pins equal to the generic one, because the generic form would take about four
times longer at 120 modes.  After each checkpoint the oracle field is sampled
at S seeded positions per mode (``--samples``) and written with the exact row
norms as ``tests/golden/<workload>_step<k>.npz``; MANIFEST.json gets the
file's sha256, the commit of the tree that wrote it, the digest of the oracle
functions on the path and the digest of the inputs (see tests/golden_store.py).
The oracle/ and workloads/ folders must be committed (clean) so that the
recorded commit names the code that computed the values.
"""

from __future__ import annotations

import argparse
import datetime
import json
import os
import subprocess
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import golden_store as G  # noqa: E402
import oracle  # noqa: E402
import workloads as W  # noqa: E402

SAMPLES = {"wdm36": 1024, "wdm120": 512}
KERR_FORM = {"wdm36": "generic", "wdm120": "packed"}


def git(*args: str) -> str:
    return subprocess.run(["git", *args], cwd=ROOT, capture_output=True, text=True, check=True).stdout.strip()


def sample_positions(M: int, T: int, n: int) -> np.ndarray:
    rng = np.random.default_rng((190101895, 77, M, T))
    return np.stack([np.sort(rng.choice(T, n, replace=False)) for _ in range(M)]).astype(np.int32)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(KERR_FORM))
    ap.add_argument("--checkpoints", type=int, nargs="+", required=True)
    ap.add_argument("--samples", type=int, default=None)
    args = ap.parse_args()
    if git("status", "--porcelain", "--", "oracle", "workloads"):
        raise SystemExit("oracle/ or workloads/ has uncommitted changes; commit them first")
    commit = git("rev-parse", "HEAD")
    p = W.make_problem(args.workload)
    n_s = args.samples or SAMPLES[args.workload]
    idx = sample_positions(p.M, p.T, n_s)
    cps = sorted(set(args.checkpoints))
    form = KERR_FORM[args.workload]
    kern = oracle.KerrGeneric(p.S, p.gamma) if form == "generic" else oracle.KerrPacked(p.S, p.gamma)
    common = {"workload": args.workload, "kerr_form": form, "M": p.M, "T": p.T, "h_km": p.h,
              "samples_per_mode": n_s, "commit": commit, "oracle_sha256": G.oracle_digest(),
              "inputs_sha256": G.inputs_digest(p)}
    t0 = time.time()

    def cb(step, A):
        if step in cps:
            name = G.file_name(args.workload, step)
            path = os.path.join(G.GOLDEN, name)
            val = np.take_along_axis(A, idx.astype(np.int64), axis=1)
            norm2 = np.sum(np.abs(A) ** 2, axis=1)
            with open(path, "wb") as f:
                np.savez(f, idx=idx, val=val.astype(np.complex128), norm2=norm2.astype(np.float64))
            man = G.manifest()
            man["files"][name] = dict(common, step=step, sha256=G.sha256_file(path),
                                      written=datetime.datetime.now(datetime.timezone.utc).isoformat(),
                                      oracle_seconds=round(time.time() - t0, 1))
            with open(G.MANIFEST, "w") as f:
                json.dump(man, f, indent=1, sort_keys=True)
                f.write("\n")
            print(f"{args.workload}: step {step} written ({time.time() - t0:.0f} s)", flush=True)
        elif step % 10 == 0:
            print(f"{args.workload}: step {step} ({time.time() - t0:.0f} s)", flush=True)

    oracle.propagate(p.A0, p.beta, None, p.S, p.gamma, p.dt, p.h, max(cps), kerr=kern, callback=cb)


if __name__ == "__main__":
    main()
