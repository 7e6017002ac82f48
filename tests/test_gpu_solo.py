"""Whole RK4IP steps of a one-mode field in one workgroup (rk4ip_solo).

A one-mode plan with 64 <= T <= 2048 (4096 with MMNLSE_SOLO=1) runs every
call's steps in one launch of one workgroup.  Its transform and Kerr arithmetic are those of the
single-pass linear kernel and the small-M Kerr kernel, in the same order, so
the field must equal bit for bit the four-launch schedule on the single-pass
transform (MMNLSE_SOLO=0, MMNLSE_FORCE_FOUR_STEP=0).  Chunked propagation
(the carried h N(A) between chunks) must equal one uninterrupted call, and
the soliton must stay within its closed-form bar (Section 2, Eq. 6).
"""

import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def _run(mm, p, n, env, monkeypatch):
    import torch
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    P = mm.Propagator.from_problem(p)
    A = torch.from_numpy(p.A0.astype(np.complex64)).cuda()
    P.advance(A, n)
    torch.cuda.synchronize()
    out = A.cpu().numpy()
    P.close()
    for k in env:
        monkeypatch.delenv(k)
    return out


@pytest.mark.parametrize("T,n", [(64, 3), (128, 5), (1024, 17), (4096, 40)])
def test_solo_matches_four_launch_schedule(gpu_lib, T, n, monkeypatch):
    """The one-workgroup side is forced (MMNLSE_SOLO=1) so that T = 4096 is
    covered too."""
    mm = gpu_lib
    p = W.soliton_problem(T=T, n_steps=n)
    print(f"solo T={T} n={n}", flush=True)
    solo = _run(mm, p, n, {"MMNLSE_SOLO": "1"}, monkeypatch)
    ref = _run(mm, p, n, {"MMNLSE_SOLO": "0", "MMNLSE_FORCE_FOUR_STEP": "0"}, monkeypatch)
    assert np.isfinite(solo).all()
    assert np.array_equal(solo, ref)


def test_solo_chunks_equal_one_call(gpu_lib, monkeypatch):
    """propagate with diagnostics every 7 steps splits the 200 steps into
    chunks that carry h N(A) (start / finish); the field is the same as
    without diagnostics."""
    import torch
    mm = gpu_lib
    monkeypatch.setenv("MMNLSE_SOLO", "1")
    p = W.make_problem("soliton")
    A0 = torch.from_numpy(p.A0.astype(np.complex64)).cuda()
    outs = []
    for diag in (0, 7):
        P = mm.Propagator.from_problem(p, diag_every=diag)
        outs.append(P.propagate(A0.clone()).cpu().numpy())
        P.close()
    assert np.array_equal(outs[0], outs[1])


def test_solo_soliton_closed_form_and_profile(gpu_lib, monkeypatch):
    """Noise-free fundamental soliton over 1 km (200 steps of 5 m): |A| keeps
    its sech shape and the phase advances by gamma P0 z / 2.  The profile
    reports the call as one Kerr-class launch holding 4 n evaluations."""
    import torch
    mm = gpu_lib
    monkeypatch.setenv("MMNLSE_SOLO", "1")
    p = W.soliton_problem(noise=0.0)
    P = mm.Propagator.from_problem(p)
    assert P.kerr_path == "small"
    A = torch.from_numpy(p.A0.astype(np.complex64)).cuda()
    prof = P.profile(A, p.n_steps)
    out = A.cpu().numpy()[0]
    P.close()
    assert prof["kerr_launches"] == 1 and prof["linear_launches"] == 0, prof
    assert prof["kerr_evals"] == 4 * p.n_steps, prof
    t = oracle.time_grid(p.T, p.dt)
    P0, T0 = p.meta["P0"], p.meta["T0"]
    exact = math.sqrt(P0) / np.cosh(t / T0) * np.exp(0.5j * p.gamma * P0 * p.L)
    err = np.linalg.norm(out - exact) / np.linalg.norm(exact)
    print(f"solo soliton rel L2 vs closed form = {err:.3e}", flush=True)
    assert err < 1e-5
