"""Degenerate and boundary inputs through the C ABI, against the oracle or
exact answers: an all-zero field, zero length, a non-finite input, the
smallest matrix-core problem (M = 3, one partly filled tile, T = 64) in all
three contraction precisions, one span equal to the whole fiber, and the
split-step with the Manakov operator on the four-step transform."""

import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_zero_field_stays_zero(gpu_lib):
    mm = gpu_lib
    p = W.make_problem("qpsk6", T=2 ** 10, n_steps=5)
    for prec in (mm.FP32, mm.SPLIT_BF16, mm.SPLIT_BF16_S):
        P = mm.Propagator.from_problem(p, precision=prec)
        out, st = P.propagate(np.zeros_like(p.A0), stats=True)
        P.close()
        assert not np.any(out) and st["power_out"] == 0.0


def test_zero_length_returns_the_input(gpu_lib):
    mm = gpu_lib
    p = W.make_problem("qpsk6", T=2 ** 10, n_steps=1)
    P = mm.Propagator.from_problem(p, L=0.0)
    out, st = P.propagate(p.A0, stats=True)
    assert st["steps"] == 0 and np.array_equal(out, p.A0)
    A128 = p.A0.astype(np.complex128) * (1 + 1e-9)
    assert np.array_equal(P.propagate(A128), A128.astype(np.complex64).astype(np.complex128))
    P.close()


def test_nonfinite_input_is_rejected_and_the_plan_survives(gpu_lib):
    mm = gpu_lib
    p = W.make_problem("qpsk6", T=2 ** 10, n_steps=2)
    P = mm.Propagator.from_problem(p)
    bad = p.A0.copy()
    bad[2, 7] = np.inf
    with pytest.raises(mm.MMNLSEError) as e:
        P.propagate(bad)
    assert e.value.status == 4
    ref = oracle.propagate(p.A0, p.beta, None, p.S, p.gamma, p.dt, p.h, p.n_steps,
                           kerr=oracle.KerrGeneric(p.S, p.gamma))
    assert rel(P.propagate(p.A0), ref) < 1e-5
    P.close()


@pytest.mark.parametrize("prec_name,tol", [("FP32", 2e-6), ("SPLIT_BF16", 3e-5), ("SPLIT_BF16_S", 3e-3)])
def test_smallest_matrix_core_problem(gpu_lib, prec_name, tol):
    """M = 3: P = 6 packed pairs in one 32-row tile (26 padding rows), T = 64."""
    mm = gpu_lib
    import torch
    M, T = 3, 64
    rng = np.random.default_rng(61)
    S = W.symmetric_gaussian_tensor(M, rng).astype(np.float32)
    P = mm.Propagator(M, T, 0.5, np.zeros((M, 1)), S, 1.3, 0.05, 0.05, precision=getattr(mm, prec_name))
    assert P.kerr_path == "mfma"
    X = ((rng.standard_normal((M, T)) + 1j * rng.standard_normal((M, T))) / math.sqrt(2)).astype(np.complex64)
    Y = P.kerr(torch.from_numpy(X).cuda()).cpu().numpy()
    ref = 0.05 * oracle.kerr_term(X.astype(np.complex128), S.astype(np.float64), 1.3)
    err = rel(Y, ref)
    print(f"M=3 T=64 {prec_name}: rel L2 = {err:.2e}", flush=True)
    assert err < tol
    P.close()


def test_one_span_over_the_whole_fiber(gpu_lib):
    """span = L: a single amplifier, after the last step."""
    mm = gpu_lib
    p = W.manakov_problem(M=6, T=2 ** 11, n_steps=10)
    kerr = oracle.KerrManakov(p.kappa.astype(np.float64), p.gamma)
    P = mm.Propagator.from_problem(p, span=p.h * p.n_steps)
    out = P.propagate(p.A0)
    P.close()
    ref = oracle.propagate(p.A0, p.beta, p.alpha, None, p.gamma, p.dt, p.h, p.n_steps, kerr=kerr,
                           span_steps=p.n_steps)
    assert rel(out, ref) < 1e-5
    Q = mm.Propagator.from_problem(p)
    plain = Q.propagate(p.A0)
    Q.close()
    g = np.exp(0.5 * p.alpha * p.h * p.n_steps).astype(np.float32)
    assert np.allclose(out, plain * g[:, None], rtol=1e-6, atol=0)


def test_agrawal_on_the_four_step_transform(gpu_lib, monkeypatch):
    mm = gpu_lib
    monkeypatch.setenv("MMNLSE_FORCE_FOUR_STEP", "1")
    p = W.manakov_problem(M=10, T=2 ** 12, n_steps=10)
    P = mm.Propagator.from_problem(p, method=mm.SSFM_AGRAWAL)
    out = P.propagate(p.A0)
    P.close()
    ref = oracle.propagate(p.A0, p.beta, p.alpha, None, p.gamma, p.dt, p.h, p.n_steps,
                           kerr=oracle.KerrManakov(p.kappa.astype(np.float64), p.gamma), method="ssfm_agrawal")
    assert rel(out, ref) < 1e-5
