"""Stored FP64-oracle reference samples for the long parity checks, and their manifest.

The oracle needs hours for the full-length wdm36 run (36 modes, T = 2^16,
1000 steps) and tens of minutes for a 5-step slice of wdm120 (120 modes,
T = 2^17), so ``tests/golden/make_golden.py`` computes them once, with
``oracle/`` only, and stores per checkpoint (step count):

    idx   [M, S] int32      sample positions t of each mode (seeded, sorted, distinct)
    val   [M, S] complex128 the oracle field A_p(t) at those positions
    norm2 [M]    float64    sum_t |A_p(t)|^2 over the whole oracle row

``tests/golden/MANIFEST.json`` records for every file its sha256, the
workload, the Kerr form the oracle used, the git commit of the tree that
wrote it, a sha256 of the oracle functions on the path and a sha256 of the
generated inputs (field, beta, S).  ``load`` checks the file's hash, and
``inputs_digest`` lets a test confirm that the inputs it regenerates are the
ones the stored values were computed from.

Error estimate from the samples: with the exact row norms and S samples of
the difference per row, ||d_p||^2 ~ (T / S) sum_samples |d_p(t)|^2, so the
relative L2 over the field is sqrt(sum_p ||d_p||^2 / sum_p norm2_p) and the
per-mode one sqrt(||d_p||^2 / norm2_p).
"""

from __future__ import annotations

import hashlib
import inspect
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
MANIFEST = os.path.join(GOLDEN, "MANIFEST.json")


def file_name(workload: str, step: int) -> str:
    return f"{workload}_step{step}.npz"


def sha256_file(path: str) -> str:
    h = hashlib.sha256()
    with open(path, "rb") as f:
        for chunk in iter(lambda: f.read(1 << 20), b""):
            h.update(chunk)
    return h.hexdigest()


def inputs_digest(p) -> str:
    """sha256 over the bytes of the problem's launch field, beta and tensor."""
    h = hashlib.sha256()
    for a in (p.A0, p.beta, p.S):
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    h.update(repr((float(p.gamma), float(p.dt), float(p.h))).encode())
    return h.hexdigest()


def oracle_digest() -> str:
    """sha256 of the source of the oracle functions the stored runs go through."""
    import oracle.rk4ip as R
    parts = [R.time_grid, R.angular_frequencies, R.linear_operator, R.half_step_propagator,
             R.apply_linear, R.KerrGeneric, R.KerrPacked, R.rk4ip_step, R.propagate, R._kerr_for]
    h = hashlib.sha256()
    for obj in parts:
        h.update(inspect.getsource(obj).encode())
    return h.hexdigest()


def manifest() -> dict:
    if not os.path.exists(MANIFEST):
        return {"files": {}}
    with open(MANIFEST) as f:
        return json.load(f)


def checkpoints(workload: str) -> list[int]:
    return sorted(int(v["step"]) for v in manifest()["files"].values() if v["workload"] == workload)


def load(workload: str, step: int) -> tuple[dict, dict]:
    """(arrays, manifest entry) of one checkpoint; raises if the file does not match its hash."""
    name = file_name(workload, step)
    entry = manifest()["files"].get(name)
    if entry is None:
        raise FileNotFoundError(f"{name} is not in {MANIFEST}")
    path = os.path.join(GOLDEN, name)
    digest = sha256_file(path)
    if digest != entry["sha256"]:
        raise ValueError(f"{name}: sha256 {digest} does not match the manifest ({entry['sha256']})")
    with np.load(path, allow_pickle=False) as z:
        arrays = {k: z[k] for k in ("idx", "val", "norm2")}
    return arrays, entry


def sample_errors(field: np.ndarray, ref: dict) -> tuple[float, np.ndarray]:
    """(relative L2 over the field, relative L2 per mode) of ``field`` [M, T]
    against stored samples ``ref``, estimated as in the module docstring."""
    idx, val, norm2 = ref["idx"], ref["val"], ref["norm2"]
    M, T = field.shape
    got = np.take_along_axis(np.asarray(field), idx.astype(np.int64), axis=1).astype(np.complex128)
    d2 = np.sum(np.abs(got - val) ** 2, axis=1) * (T / idx.shape[1])
    return float(np.sqrt(d2.sum() / norm2.sum())), np.sqrt(d2 / norm2)
