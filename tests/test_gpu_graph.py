"""Replayed step graphs for launch-bound plans.

mmnlse_advance and mmnlse_propagate run the middle steps of a small plan as
a captured HIP graph.  The graph holds the same kernels with the same
arguments as the eager schedule, so every replay must reproduce the eager
result bit for bit; replays are interleaved with other eager work and
synchronisations, and a new field pointer triggers a new capture.
"""

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def _eager(mm, p, n, monkeypatch):
    import torch
    monkeypatch.setenv("MMNLSE_GRAPH", "0")
    P = mm.Propagator.from_problem(p)
    A = torch.from_numpy(p.A0.astype(np.complex64)).cuda()
    P.advance(A, n)
    torch.cuda.synchronize()
    P.close()
    monkeypatch.delenv("MMNLSE_GRAPH")
    return A.cpu().numpy()


@pytest.mark.parametrize("name,kw", [("qpsk6", dict(T=2 ** 12, n_steps=1)), ("soliton", dict(n_steps=1))])
def test_graph_replays_match_eager(gpu_lib, name, kw, monkeypatch):
    import torch
    mm = gpu_lib
    p = W.make_problem(name, **kw)
    n = 40                                   # first step, 2 graph replays of 16, 7 more
    ref = _eager(mm, p, n, monkeypatch)
    A0 = torch.from_numpy(p.A0.astype(np.complex64)).cuda()
    P = mm.Propagator.from_problem(p)
    A = A0.clone()
    P.advance(A, 1)                          # a short call first (captures, runs eagerly)
    for rep in range(3):
        A.copy_(A0)
        P.advance(A, n)
        torch.cuda.synchronize()
        assert np.array_equal(A.cpu().numpy(), ref), f"replay {rep}"
        X = P.linear_half_step(A)            # unrelated eager work between replays
        torch.cuda.synchronize()
        assert np.isfinite(X.cpu().numpy()).all()
    B = A0.clone()                           # a new pointer: captured again
    P.advance(B, n)
    torch.cuda.synchronize()
    assert np.array_equal(B.cpu().numpy(), ref)
    P.close()


def test_graph_propagation_matches_oracle(gpu_lib):
    mm = gpu_lib
    p = W.make_problem("qpsk6", T=2 ** 12, n_steps=60)
    P = mm.Propagator.from_problem(p)
    P.propagate(p.A0)                        # warm
    out = P.propagate(p.A0)
    ref = oracle.propagate(p.A0, p.beta, None, p.S, p.gamma, p.dt, p.h, p.n_steps,
                           kerr=oracle.KerrGeneric(p.S, p.gamma))
    err = float(np.linalg.norm(out - ref) / np.linalg.norm(ref))
    print(f"qpsk6 T=2^12, 60 steps through the graph path: rel L2 {err:.3e}", flush=True)
    assert err < 1e-5
    P.close()
