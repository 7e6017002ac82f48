"""Serving (continuous batching) on the GPU through the C-ABI.

A request's result must be bit-identical alone (mmnlse_propagate) and in any
mix of concurrently resident requests: every request owns its plan and work
fields, kernels are deterministic (no atomics), and the step schedule carries
h N(A) across scheduling rounds.
"""

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def mixed_requests(mm):
    reqs = []
    specs = [("qpsk6", 1, 2 ** 10, 5), ("qpsk6", 6, 2 ** 12, 7), ("qpsk6", 3, 2 ** 15, 3),
             ("wdm36", 12, 2 ** 11, 4), ("qpsk6", 6, 2 ** 10, 11), ("wdm36", 9, 2 ** 12, 2),
             ("qpsk6", 2, 2 ** 12, 0), ("qpsk6", 4, 2 ** 13, 9)]
    for i, (style, M, T, n) in enumerate(specs):
        p = W.make_problem(style, T=T, n_steps=max(n, 1), M=M)
        L = p.h * n
        prec = mm.SPLIT_BF16 if (style == "wdm36" and i == 5) else mm.FP32
        reqs.append((p, L, prec))
    return reqs


def alone(mm, p, L, prec):
    P = mm.Propagator.from_problem(p, precision=prec, L=L)
    out = P.propagate(p.A0)
    P.close()
    return out


def test_results_identical_alone_and_in_mix(gpu_lib):
    mm = gpu_lib
    reqs = mixed_requests(mm)
    ref = [alone(mm, p, L, prec) for p, L, prec in reqs]
    with mm.Server(n_streams=3, steps_per_tick=3) as srv:
        tickets = [srv.submit(p.A0, mm.problem_config(p, precision=prec, L=L)) for p, L, prec in reqs]
        outs = [srv.wait(t) for t in tickets]
        c = srv.counters()
    for (out, info), r, (p, L, prec) in zip(outs, ref, reqs):
        assert np.array_equal(out, r), p.name
        assert info["steps"] == int(round(L / p.h))
        assert info["latency"] > 0
    assert c["completed"] == len(reqs) and c["failed"] == 0 and c["queued"] == 0


def test_small_budget_admits_one_at_a_time(gpu_lib):
    mm = gpu_lib
    reqs = mixed_requests(mm)[:4]
    ref = [alone(mm, p, L, prec) for p, L, prec in reqs]
    # largest single footprint is ~6 MB here; 12 MB cannot hold two large ones
    budget = 12 * 2 ** 20
    with mm.Server(mem_budget_bytes=budget, n_streams=2, steps_per_tick=2) as srv:
        tickets = [srv.submit(p.A0, mm.problem_config(p, precision=prec, L=L)) for p, L, prec in reqs]
        outs = [srv.wait(t)[0] for t in tickets]
        c = srv.counters()
    for o, r in zip(outs, ref):
        assert np.array_equal(o, r)
    assert 0 < c["peak_admitted_bytes"] <= budget


def test_served_soliton_matches_oracle(gpu_lib):
    mm = gpu_lib
    p = W.make_problem("soliton")
    with mm.Server() as srv:
        t = srv.submit(p.A0, mm.problem_config(p))
        out, info = srv.wait(t)
    ref = oracle.propagate(p.A0, p.beta, None, p.S, p.gamma, p.dt, p.h, p.n_steps)
    assert out.dtype == np.complex128
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 1e-5
    assert abs(info["power_out"] / info["power_in"] - 1) < 1e-5


def test_error_paths_leave_server_usable(gpu_lib):
    mm = gpu_lib
    p = W.make_problem("qpsk6", T=2 ** 10, n_steps=2)
    with mm.Server(mem_budget_bytes=2 ** 20) as srv:
        big = W.make_problem("qpsk6", T=2 ** 14, n_steps=1)
        with pytest.raises(mm.MMNLSEError) as e:
            srv.submit(big.A0, mm.problem_config(big))
        assert e.value.status == 2  # E_NOMEM: can never fit
        with pytest.raises(mm.MMNLSEError) as e:
            srv.submit(p.A0, mm.problem_config(p, L=p.h * 2.5))
        assert e.value.status == 1  # E_INVALID: L/h not an integer
        bad = p.A0.copy()
        bad[0, 3] = np.nan
        tb = srv.submit(bad, mm.problem_config(p))
        with pytest.raises(mm.MMNLSEError) as e:
            srv.wait(tb)
        assert e.value.status == 4  # E_NONFINITE
        with pytest.raises(mm.MMNLSEError):
            srv.poll(123456)
        t = srv.submit(p.A0, mm.problem_config(p))
        out, _ = srv.wait(t)
        assert np.array_equal(out, alone(mm, p, p.L, mm.FP32))
        assert srv.counters()["failed"] == 1


def test_spans_and_manakov_requests_served_like_alone(gpu_lib):
    """Requests with amplified spans (rounds of 4 steps against spans of 3 and
    5) and with the Manakov operator: bit-identical to a lone propagation."""
    import dataclasses
    mm = gpu_lib
    man = W.manakov_problem(M=30, T=2 ** 12, n_steps=20)
    q = dataclasses.replace(W.make_problem("qpsk6", T=2 ** 11, n_steps=9), alpha=np.full(6, 0.2))
    reqs = [(man, 5 * man.h), (q, 3 * q.h), (man, 0.0)]
    ref = []
    for p, span in reqs:
        P = mm.Propagator.from_problem(p, span=span)
        ref.append(P.propagate(p.A0))
        P.close()
    with mm.Server(n_streams=2, steps_per_tick=4) as srv:
        tickets = [srv.submit(p.A0, mm.problem_config(p, span=span)) for p, span in reqs]
        outs = [srv.wait(t)[0] for t in tickets]
    for o, r in zip(outs, ref):
        assert np.array_equal(o, r)


def test_agrawal_requests_served_like_alone(gpu_lib):
    """SSFM-Agrawal on the four-step transform (M = 30 rows, T = 2^12) shares
    the last half step of a step with the first of the next; the server's
    ticks (3 steps) and a span end (every 5 steps) carry or restart that
    shared transform exactly as one propagation does: bit-identical results,
    and so are propagations with diagnostics every 4 steps."""
    mm = gpu_lib
    man = W.manakov_problem(M=30, T=2 ** 12, n_steps=20)
    reqs = [(man, 0.0), (man, 5 * man.h)]
    ref = []
    for p, span in reqs:
        P = mm.Propagator.from_problem(p, method=mm.SSFM_AGRAWAL, span=span)
        ref.append(P.propagate(p.A0))
        P.close()
        P = mm.Propagator.from_problem(p, method=mm.SSFM_AGRAWAL, span=span, diag_every=4)
        assert np.array_equal(P.propagate(p.A0), ref[-1])
        P.close()
    with mm.Server(n_streams=2, steps_per_tick=3) as srv:
        tickets = [srv.submit(p.A0, mm.problem_config(p, method=mm.SSFM_AGRAWAL, span=span)) for p, span in reqs]
        outs = [srv.wait(t)[0] for t in tickets]
    for o, r in zip(outs, ref):
        assert np.array_equal(o, r)
