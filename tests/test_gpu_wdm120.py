"""Parity at the largest workload, wdm120 (M=120 modes, T=2^17, dense symmetric S).

At full size the FP64 oracle cannot run whole steps in test time, so:
  * the Kerr increment of the full field is compared on sampled time columns
    (the Kerr term is pointwise in t, so the oracle evaluates just those);
  * the half-step propagator of the full field is compared on sampled rows
    (it acts on each mode's row independently);
  * a whole propagation is compared at reduced T (same M, tensor and beta);
  * over a few full-size steps, the FP32 and split-bf16 paths must agree.
"""

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def wdm120():
    print("generating wdm120", flush=True)
    return W.make_problem("wdm120")


@pytest.mark.parametrize("precision,tol", [("fp32", 2e-6), ("split_bf16", 3e-5)])
def test_wdm120_kerr_on_sampled_columns(gpu_lib, wdm120, precision, tol):
    import torch
    mm = gpu_lib
    p = wdm120
    P = mm.Propagator.from_problem(p, precision=mm.FP32 if precision == "fp32" else mm.SPLIT_BF16)
    assert P.kerr_path == "mfma"
    X = torch.from_numpy(p.A0).cuda()
    Y = P.kerr(X).cpu().numpy()
    cols = np.random.default_rng(120).choice(p.T, 48, replace=False)
    ref = p.h * oracle.KerrPacked(p.S, p.gamma)(p.A0[:, cols].astype(np.complex128))
    err = rel(Y[:, cols], ref)
    print(f"wdm120 kerr {precision}: rel L2 on {cols.size} columns = {err:.3e}", flush=True)
    assert err < tol
    P.close()


def test_wdm120_linear_on_sampled_rows(gpu_lib, wdm120):
    import torch
    mm = gpu_lib
    p = wdm120
    P = mm.Propagator.from_problem(p)
    Y = P.linear_half_step(torch.from_numpy(p.A0).cuda()).cpu().numpy()
    rows = [0, 17, 64, 119]
    E = oracle.half_step_propagator(oracle.angular_frequencies(p.T, p.dt), p.beta[rows], None, p.h)
    ref = oracle.apply_linear(p.A0[rows].astype(np.complex128), E)
    assert rel(Y[rows], ref) < 1e-6
    P.close()


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("split_bf16", 1e-4)])
def test_wdm120_reduced_T_propagation(gpu_lib, wdm120, precision, tol):
    mm = gpu_lib
    p = W.make_problem("wdm120", T=2 ** 11, n_steps=2, tensor=(wdm120.S, wdm120.meta))
    P = mm.Propagator.from_problem(p, precision=mm.FP32 if precision == "fp32" else mm.SPLIT_BF16)
    out = P.propagate(p.A0)
    ref = oracle.propagate(p.A0, p.beta, None, p.S, p.gamma, p.dt, p.h, p.n_steps,
                           kerr=oracle.KerrPacked(p.S, p.gamma))
    err = rel(out, ref)
    print(f"wdm120 T=2^11 {precision}: rel L2 = {err:.3e}", flush=True)
    assert err < tol
    P.close()


def test_wdm120_full_size_fp32_and_split_agree(gpu_lib, wdm120):
    import torch
    mm = gpu_lib
    p = wdm120
    outs = {}
    for name, prec in (("fp32", mm.FP32), ("split", mm.SPLIT_BF16)):
        P = mm.Propagator.from_problem(p, precision=prec)
        A = torch.from_numpy(p.A0).cuda()
        P.advance(A, 5)
        torch.cuda.synchronize()
        outs[name] = A.cpu().numpy()
        pin, pout = P.power(torch.from_numpy(p.A0).cuda()), P.power(A)
        print(f"wdm120 {name}: 5 steps, power drift {pout / pin - 1:.2e}", flush=True)
        P.close()
    d = rel(outs["split"], outs["fp32"])
    print(f"wdm120 split vs fp32 after 5 full-size steps: {d:.3e}", flush=True)
    assert d < 1e-4
