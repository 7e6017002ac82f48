"""The allocation-free power entry point (mmnlse_power_noalloc) against
mmnlse_power, called through the C ABI on two calls in a row, the second on a
smaller field.  Both run the same FP64 reduction with the same blocks and
summation order, so the values must be identical; each is also checked
against the FP64 oracle's power (dt * sum |A|^2)."""

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def test_power_noalloc_matches_power_on_two_calls(gpu_lib):
    import torch
    mm = gpu_lib
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    cases = [W.make_problem("qpsk6", T=2 ** 16),         # 393216 values: 96 partials
             W.make_problem("soliton", T=2 ** 12)]        # 4096 values: 1 partial
    seen = []
    for p in cases:
        print(f"power_noalloc: {p.name} M={p.M} T={p.T}", flush=True)
        A = np.ascontiguousarray(p.A0.astype(np.complex64))
        X = torch.from_numpy(A).cuda()
        P = mm.Propagator.from_problem(p)
        ref = P.power(X)
        P.close()
        mm.power_noalloc(X, p.dt, out)
        torch.cuda.synchronize()
        got = float(out.item())
        assert got == ref, (got, ref)
        exact = oracle.power(A.astype(np.complex128), p.dt)
        assert abs(got / exact - 1.0) < 1e-12, (got, exact)
        seen.append(got)
    assert seen[0] != seen[1]


def test_power_noalloc_on_a_side_stream(gpu_lib):
    import torch
    mm = gpu_lib
    p = W.make_problem("qpsk6", T=2 ** 12)
    X = torch.from_numpy(p.A0).cuda()
    s = torch.cuda.Stream()
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        mm.power_noalloc(X, p.dt, out, stream=s)
    s.synchronize()
    P = mm.Propagator.from_problem(p)
    assert float(out.item()) == P.power(X)
    P.close()


def test_power_noalloc_rejects_bad_sizes(gpu_lib):
    import ctypes
    import torch
    mm = gpu_lib
    lib = mm.load()
    X = torch.zeros(64, dtype=torch.complex64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    xp, op = ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(out.data_ptr())
    for n, dt in ((0, 1.0), (-5, 1.0), ((1 << 40) + 1, 1.0), (64, 0.0), (64, float("inf"))):
        assert lib.mmnlse_power_noalloc(xp, n, dt, op, None) == 1, (n, dt)
        assert lib.mmnlse_last_error()
    assert lib.mmnlse_power_noalloc(None, 64, 1.0, op, None) == 1
