"""Input generators: shapes, seeds, symmetry and the stated recipe (CPU only)."""

import numpy as np

import workloads as W


def test_qpsk6_shapes_power_and_tensor():
    p = W.make_problem("qpsk6")
    assert p.A0.shape == (6, 2 ** 14) and p.A0.dtype == np.complex64
    assert abs(p.dt - 31.25 / 8) < 1e-15
    np.testing.assert_allclose(np.mean(np.abs(p.A0) ** 2, axis=1), 1e-3, rtol=1e-5)
    S = p.S.astype(np.float64)
    for perm in [(1, 0, 2, 3), (0, 2, 1, 3), (3, 1, 2, 0), (2, 3, 0, 1)]:
        assert np.array_equal(S, S.transpose(perm))
    assert np.abs(S).max() == 1.0
    assert p.n_steps == 100 and abs(p.L - 10.0) < 1e-12
    assert np.all(p.beta[:, 2] <= -15) and np.all(p.beta[:, 2] >= -25)
    assert np.all(np.abs(p.beta[:, 1]) <= 500)


def test_seeded_and_reproducible():
    a = W.make_problem("qpsk6", T=1024)
    b = W.make_problem("qpsk6", T=1024)
    assert np.array_equal(a.A0, b.A0) and np.array_equal(a.S, b.S) and np.array_equal(a.beta, b.beta)


def test_wdm36_mask_fraction_and_pure_classes_kept():
    p = W.make_problem("wdm36", T=2 ** 11)
    assert 0.70 <= p.meta["zero_fraction"] < 0.75
    g = W.mode_groups(36)
    assert g.max() == 7
    # every (g,g,g,g) class survives, so self-phase modulation stays on
    ar = np.arange(36)
    assert np.all(p.S[ar, ar, ar, ar] != 0)
    assert np.array_equal(p.S, p.S.transpose(1, 0, 2, 3))
    np.testing.assert_allclose(np.mean(np.abs(p.A0) ** 2, axis=1), 8 * 1e-3 * 10 ** -0.2, rtol=1e-4)


def test_soliton_parameters():
    p = W.make_problem("soliton")
    assert p.A0.dtype == np.complex128 and p.A0.shape == (1, 4096)
    assert abs(p.meta["P0"] - 20.0 / (1.3 * 4.0)) < 1e-12
    assert p.n_steps == 200 and abs(p.h - 0.005) < 1e-15


def test_table3_groups():
    b = W.table3_beta(120)
    g = W.mode_groups(120)
    assert np.bincount(g).tolist() == list(range(1, 16))
    assert b[0, 1] == 0.0 and b[-1, 1] == -8.61 and b[-1, 2] == -27.4


def test_serving_stream():
    s = W.serving_stream(256)
    assert len(s) == 256
    assert {r.M for r in s} <= {1, 6, 15, 36}
    assert {r.T for r in s} <= {2 ** 12, 2 ** 14, 2 ** 16}
    r = W.serving_stream(8, rate=10.0)
    assert all(b.arrival >= a.arrival for a, b in zip(r, r[1:]))
