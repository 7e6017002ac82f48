"""Write FP64-oracle reference fields for the long parity checks.

    python tests/golden/make_golden.py wdm36 --checkpoints 10 30 100 300 1000
    python tests/golden/make_golden.py wdm120 --checkpoints 1 5

Runs only ``oracle/`` on inputs from ``workloads/`` and stores the oracle
field after the given step counts as complex64 ``.npy`` files under
tests/golden/cache/ (git-ignored: tens of MB each).  complex64 storage adds
at most 6e-8 relative error, far below the 1e-5 / 1e-4 parity bars.
"""

from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

CACHE = os.path.join(HERE, "cache")


def path_for(name: str, steps: int) -> str:
    return os.path.join(CACHE, f"{name}_oracle_step{steps}.npy")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--checkpoints", type=int, nargs="+", required=True)
    args = ap.parse_args()
    os.makedirs(CACHE, exist_ok=True)
    p = W.make_problem(args.workload)
    cps = sorted(set(args.checkpoints))
    kern = oracle.KerrPacked(p.S, p.gamma) if p.symmetric else oracle.KerrGeneric(p.S, p.gamma)
    t0 = time.time()

    def cb(step, A):
        if step in cps:
            np.save(path_for(p.name, step), A.astype(np.complex64))
            print(f"{p.name}: step {step} saved ({time.time() - t0:.0f} s)", flush=True)
        elif step % 10 == 0:
            print(f"{p.name}: step {step} ({time.time() - t0:.0f} s)", flush=True)

    oracle.propagate(p.A0, p.beta, None, p.S, p.gamma, p.dt, p.h, max(cps), kerr=kern, callback=cb)


if __name__ == "__main__":
    main()
