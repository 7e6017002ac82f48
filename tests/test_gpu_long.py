"""Full-length parity on the wdm36 workload (M=36, T=2^16, h=50 m, 1000 steps).

The FP64 oracle needs hours for this run, so its fields are precomputed at a few
step counts by tests/golden/make_golden.py (which calls only oracle/) into
tests/golden/cache/; this test is skipped when that cache is absent.  The GPU
run is one uninterrupted step schedule with snapshots taken between segments.
Bars: relative L2 <= 1e-5 (FP32 path) and <= 1e-4 (both split-bf16 paths).
"""

import glob
import os
import re

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cache")


def checkpoints(name):
    out = {}
    for f in glob.glob(os.path.join(CACHE, f"{name}_oracle_step*.npy")):
        out[int(re.search(r"step(\d+)\.npy$", f).group(1))] = f
    return dict(sorted(out.items()))


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("split_bf16", 1e-4), ("split_bf16_s", 1e-4)])
def test_wdm36_full_length(gpu_lib, precision, tol):
    import torch
    mm = gpu_lib
    cps = checkpoints("wdm36")
    if not cps:
        pytest.skip("no cached oracle fields (run tests/golden/make_golden.py wdm36 ...)")
    p = W.make_problem("wdm36")
    prec = {"fp32": mm.FP32, "split_bf16": mm.SPLIT_BF16, "split_bf16_s": mm.SPLIT_BF16_S}[precision]
    P = mm.Propagator.from_problem(p, precision=prec)
    A = torch.from_numpy(p.A0).cuda()
    done, errs = 0, {}
    for s, f in cps.items():
        P.advance(A, s - done)
        done = s
        torch.cuda.synchronize()
        ref = np.load(f).astype(np.complex128)
        got = A.cpu().numpy().astype(np.complex128)
        errs[s] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        print(f"wdm36 {precision} step {s}: rel L2 = {errs[s]:.3e}", flush=True)
    P.close()
    assert max(errs.values()) < tol, errs
