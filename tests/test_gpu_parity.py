"""GPU parity: the HIP path through the C-ABI vs the FP64 oracle on the same inputs.

Tolerances (relative L2 over all M*T complex values):
  * one half-step propagator application: 1e-6.  An FP32 FFT pair of size T
    rounds each value about 2*log2(T) times at unit roundoff 6e-8, which is
    ~5e-7 in the worst case here (T = 2^17), random in sign.
  * one Kerr evaluation: 2e-6 (FP32 products and sums over M^3 terms).
  * whole propagation, FP32 path: 1e-5 (the stated bar of the method's FP32
    path against the FP64 reference).
"""

import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def crandn(rng, *shape):
    return ((rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2)).astype(np.complex64)


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(x):
    return x.cpu().numpy()


def make(mm, M, T, dt=0.5, beta=None, S=None, gamma=1.0, h=0.1, L=0.1, seed=0, **kw):
    rng = np.random.default_rng((7, M, T, seed))
    if beta is None:
        beta = np.column_stack([rng.uniform(-50, 50, M), rng.uniform(-20, 20, M), rng.uniform(-25, -15, M)])
    if S is None:
        S = W.symmetric_gaussian_tensor(M, rng).astype(np.float32)
    return mm.Propagator(M, T, dt, beta, S, gamma, h, L, **kw), beta, S


@pytest.mark.parametrize("T", [64, 256, 1024, 4096, 16384, 2 ** 15, 2 ** 16, 2 ** 17])
def test_linear_half_step(gpu_lib, T, monkeypatch):
    """One-pass LDS FFT for every T <= 2^14 (forced), four-step above."""
    monkeypatch.setenv("MMNLSE_FORCE_FOUR_STEP", "0")
    mm = gpu_lib
    M = 3
    print(f"linear_half_step T={T}", flush=True)
    P, beta, S = make(mm, M, T)
    rng = np.random.default_rng((11, T))
    X = crandn(rng, M, T)
    Y = host(P.linear_half_step(dev(X)))
    E = oracle.half_step_propagator(oracle.angular_frequencies(T, P.dt), beta, None, P.h)
    ref = oracle.apply_linear(X.astype(np.complex128), E)
    assert rel(Y, ref) < 1e-6
    P.close()


@pytest.mark.parametrize("T", [1024, 4096, 16384])
def test_linear_half_step_four_step_forced(gpu_lib, T, monkeypatch):
    monkeypatch.setenv("MMNLSE_FORCE_FOUR_STEP", "1")
    mm = gpu_lib
    print(f"linear_half_step four-step T={T}", flush=True)
    P, beta, S = make(mm, 5, T, seed=1)
    X = crandn(np.random.default_rng((12, T)), 5, T)
    Y = host(P.linear_half_step(dev(X)))
    E = oracle.half_step_propagator(oracle.angular_frequencies(T, P.dt), beta, None, P.h)
    assert rel(Y, oracle.apply_linear(X.astype(np.complex128), E)) < 1e-6
    P.close()


def test_linear_with_attenuation(gpu_lib):
    mm = gpu_lib
    M, T = 2, 1024
    beta = np.array([[1.0, 2.0, -20.0, 0.5], [0.0, -3.0, -10.0, 0.0]])
    alpha = np.array([0.3, 0.05])
    S = np.zeros((M,) * 4, np.float32)
    P = mm.Propagator(M, T, 0.3, beta, S, 0.0, 0.2, 0.2, alpha=alpha)
    X = crandn(np.random.default_rng(3), M, T)
    Y = host(P.linear_half_step(dev(X)))
    E = oracle.half_step_propagator(oracle.angular_frequencies(T, 0.3), beta, alpha, 0.2)
    assert rel(Y, oracle.apply_linear(X.astype(np.complex128), E)) < 1e-6
    P.close()


@pytest.mark.parametrize("M,sym,generic,path", [
    (1, True, False, "small"), (2, False, False, "small"), (2, True, False, "small"),
    (6, True, False, "small"), (8, False, False, "small"), (5, False, True, "tiled"),
    (12, True, True, "tiled"), (13, False, False, "tiled"),
    (3, True, False, "mfma"), (6, True, False, "mfma"),
    (9, True, False, "mfma"), (12, True, False, "mfma"), (36, True, False, "mfma"),
    (70, True, False, "mfma")])
def test_kerr_term(gpu_lib, M, sym, generic, path, monkeypatch):
    mm = gpu_lib
    T = 512
    if path == "small" and sym and M > 2:
        monkeypatch.setenv("MMNLSE_KERR_PATH", "0")  # keep the register kernel covered
    print(f"kerr M={M} sym={sym} generic={generic}", flush=True)
    rng = np.random.default_rng((13, M))
    S = (W.symmetric_gaussian_tensor(M, rng) if sym else rng.standard_normal((M,) * 4)).astype(np.float32)
    P, beta, S = make(mm, M, T, S=S, gamma=1.3, h=0.05, L=0.05, generic=generic)
    assert P.kerr_path == path
    X = crandn(rng, M, T)
    Y = host(P.kerr(dev(X)))
    ref = 0.05 * oracle.kerr_term(X.astype(np.complex128), S.astype(np.float64), 1.3)
    assert rel(Y, ref) < 2e-6, P.kerr_path
    P.close()


@pytest.mark.parametrize("M", [9, 36])
def test_kerr_term_split_bf16_s(gpu_lib, M):
    """Two-product contraction: S as bf16 hi + lo, B = X_l X_m rounded once to
    bf16 (relative error <= 2^-9 per product).  One evaluation is ~1.7e-3
    from the FP64 value (a CPU model of that rounding gives 1.69e-3 / 1.67e-3
    for these inputs), and the three-product path is far closer."""
    mm = gpu_lib
    T = 512
    rng = np.random.default_rng((14, M))
    S = W.symmetric_gaussian_tensor(M, rng).astype(np.float32)
    X = crandn(rng, M, T)
    ref = 0.05 * oracle.kerr_term(X.astype(np.complex128), S.astype(np.float64), 1.3)
    errs = {}
    for prec in (mm.SPLIT_BF16, mm.SPLIT_BF16_S):
        P, beta, _ = make(mm, M, T, S=S, gamma=1.3, h=0.05, L=0.05, precision=prec)
        assert P.kerr_path == "mfma"
        errs[prec] = rel(host(P.kerr(dev(X))), ref)
        P.close()
    print(f"M={M}: three products {errs[mm.SPLIT_BF16]:.2e}, two {errs[mm.SPLIT_BF16_S]:.2e}", flush=True)
    assert 1e-3 < errs[mm.SPLIT_BF16_S] < 2.5e-3
    assert errs[mm.SPLIT_BF16] < 3e-5


@pytest.mark.parametrize("M", [9, 36])
def test_kerr_term_split_bf16(gpu_lib, M):
    """Split-bf16 contraction: S and B = X_l X_m each carried as bf16 hi + lo, three
    products accumulated in FP32; each product keeps ~16 significant bits, so one
    evaluation lands within ~1e-5 of the FP64 value."""
    mm = gpu_lib
    T = 512
    rng = np.random.default_rng((14, M))
    S = W.symmetric_gaussian_tensor(M, rng).astype(np.float32)
    P, beta, S = make(mm, M, T, S=S, gamma=1.3, h=0.05, L=0.05, precision=mm.SPLIT_BF16)
    assert P.kerr_path == "mfma"
    X = crandn(rng, M, T)
    Y = host(P.kerr(dev(X)))
    ref = 0.05 * oracle.kerr_term(X.astype(np.complex128), S.astype(np.float64), 1.3)
    assert rel(Y, ref) < 3e-5
    P.close()


def _arranged_tiles(mm, S, split):
    """(tiles, tiles whose slot pairs 8g + j / 8g + 4 + j differ in p and n)."""
    M = S.shape[0]
    na, nb = [], []
    for i in range(M):
        for j in range(i, M):
            na.append(i)
            nb.append(j)
    rows = np.asarray(mm.kerr_plan(S, split)["rows"]).reshape(-1, 32)
    ok = 0
    for t in range(rows.shape[0]):
        pairs = [(rows[t, 8 * g + j], rows[t, 8 * g + 4 + j]) for g in range(4) for j in range(4)]
        ok += all(x < 0 or y < 0 or (na[x] != na[y] and nb[x] != nb[y]) for x, y in pairs)
    return rows.shape[0], ok


@pytest.mark.parametrize("kernel", ["pass", "group"])
@pytest.mark.parametrize("tensor", ["dense20", "dense36", "masked28"])
def test_kerr_contraction_kernels_and_scatters(gpu_lib, kernel, tensor, monkeypatch):
    """Both matrix-core kernels forced on dense and mode-group-masked tensors,
    in all three precisions, against the oracle's definition.  The per-pass
    kernel scatters tiles whose rows the plan could place for both lane halves
    at once together and the others in turns; the dense 20- and 36-mode plans
    hold both kinds (checked on the host), the masked one only the first."""
    mm = gpu_lib
    M = int(tensor[-2:])
    T = 512
    rng = np.random.default_rng((15, M))
    if tensor.startswith("dense"):
        S = W.symmetric_gaussian_tensor(M, rng).astype(np.float32)
    else:
        S, _ = W.fiber.coupling_tensor(M, 7, mask_frac=0.7)
    for split in (0, 1):
        tiles, ok = _arranged_tiles(mm, S, split)
        if tensor.startswith("dense"):
            assert 0 < ok < tiles, (tiles, ok)
        else:
            assert ok == tiles, (tiles, ok)
    monkeypatch.setenv("MMNLSE_GROUP_KERNEL", "0" if kernel == "pass" else "1")
    X = crandn(rng, M, T)
    ref = 0.05 * oracle.kerr_term(X.astype(np.complex128), S.astype(np.float64), 1.3)
    # two products: B rounded once to bf16 (2^-9 relative per product, unbiased)
    for prec, lo, hi in ((mm.FP32, 0.0, 2e-6), (mm.SPLIT_BF16, 0.0, 3e-5), (mm.SPLIT_BF16_S, 5e-4, 3e-3)):
        P, _, _ = make(mm, M, T, S=S, gamma=1.3, h=0.05, L=0.05, precision=prec, symmetric=True)
        assert P.kerr_path == "mfma"
        err = rel(host(P.kerr(dev(X))), ref)
        print(f"{kernel} {tensor} precision {prec}: rel L2 {err:.2e}", flush=True)
        assert lo <= err < hi, (prec, err)
        P.close()


def test_power_reduction(gpu_lib):
    mm = gpu_lib
    P, _, _ = make(mm, 4, 4096)
    X = crandn(np.random.default_rng(5), 4, 4096)
    assert abs(P.power(dev(X)) / oracle.power(X, P.dt) - 1) < 1e-12
    P.close()


_REFS = {}


def _oracle_field(p):
    """The oracle's field after the problem's steps, generic Kerr form (the
    plain definition: no symmetry of S used); computed once per problem."""
    key = (p.name, p.M, p.T, p.n_steps)
    if key not in _REFS:
        _REFS[key] = oracle.propagate(p.A0, p.beta, None, p.S, p.gamma, p.dt, p.h, p.n_steps,
                                      kerr=oracle.KerrGeneric(p.S, p.gamma))
    return _REFS[key]


def per_mode_rel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def _propagate_parity(mm, p, tol, **kw):
    print(f"propagate {p.name} M={p.M} T={p.T} steps={p.n_steps} {kw}", flush=True)
    P = mm.Propagator.from_problem(p, **kw)
    out, st = P.propagate(p.A0, stats=True)
    ref = _oracle_field(p)
    err = rel(out, ref)
    worst = float(per_mode_rel(out, ref).max())
    print(f"  rel L2 = {err:.3e}, worst mode {worst:.3e}  kerr path = {P.kerr_path}", flush=True)
    assert err < tol
    # every mode within the bar, not only the field as a whole
    assert worst < tol
    assert st["steps"] == p.n_steps
    assert abs(st["power_in"] / oracle.power(p.A0.astype(np.complex64), p.dt) - 1) < 1e-12
    P.close()
    return out, ref, st


def test_soliton_full(gpu_lib):
    p = W.make_problem("soliton")
    out, ref, st = _propagate_parity(gpu_lib, p, 1e-5)
    assert out.dtype == np.complex128
    # power conserved by the GPU path to the FP32 level
    assert abs(st["power_out"] / st["power_in"] - 1) < 1e-5


def test_qpsk6_reduced(gpu_lib):
    _propagate_parity(gpu_lib, W.make_problem("qpsk6", T=2 ** 12, n_steps=20), 1e-5)


def test_qpsk6_full(gpu_lib):
    _propagate_parity(gpu_lib, W.make_problem("qpsk6"), 1e-5)


def test_wdm36_reduced_tiled(gpu_lib):
    _propagate_parity(gpu_lib, W.make_problem("wdm36", T=2 ** 11, n_steps=4), 1e-5, generic=True)


def test_wdm36_reduced_mfma(gpu_lib):
    _propagate_parity(gpu_lib, W.make_problem("wdm36", T=2 ** 12, n_steps=20), 1e-5)


def test_wdm36_reduced_split_bf16(gpu_lib):
    import paper_1901_01895_amd as mm
    _propagate_parity(gpu_lib, W.make_problem("wdm36", T=2 ** 12, n_steps=20), 1e-4,
                      precision=mm.SPLIT_BF16)


def test_wdm36_reduced_split_bf16_s(gpu_lib):
    """Two-product mode: the bf16 rounding of B = X_l X_m leaves ~1e-5 after
    20 steps (a CPU model of that rounding gives 7.5e-6 after 10 and 1.3e-5
    after 30 steps), an order of magnitude under the 1e-4 bar."""
    import paper_1901_01895_amd as mm
    _propagate_parity(gpu_lib, W.make_problem("wdm36", T=2 ** 12, n_steps=20), 4e-5,
                      precision=mm.SPLIT_BF16_S)


def test_four_step_propagation(gpu_lib):
    p = W.make_problem("qpsk6", T=2 ** 15, n_steps=6, M=3)
    _propagate_parity(gpu_lib, p, 1e-5)


def test_device_path_and_advance_match_host_path(gpu_lib):
    import torch
    mm = gpu_lib
    p = W.make_problem("qpsk6", T=2 ** 12, n_steps=10)
    P = mm.Propagator.from_problem(p)
    out_host = P.propagate(p.A0)
    out_dev = host(P.propagate(dev(p.A0)))
    A = dev(p.A0)
    P.advance(A, p.n_steps)
    torch.cuda.synchronize()
    assert np.array_equal(out_host, out_dev)
    assert np.array_equal(out_host, host(A))
    # checkpoint / resume: two halves equal the whole, bit for bit
    B = dev(p.A0)
    P.advance(B, 4)
    P.advance(B, 6)
    torch.cuda.synchronize()
    assert np.array_equal(out_host, host(B))
    P.close()


def test_step_doubling_estimate(gpu_lib):
    mm = gpu_lib
    p = W.soliton_problem(noise=0.0, h=0.04, n_steps=1)
    P = mm.Propagator.from_problem(p)
    d_gpu = P.step_doubling(dev(p.A0.astype(np.complex64)))
    d_orc, _ = oracle.step_doubling_estimate(p.A0, p.beta, None, p.S, p.gamma, p.dt, p.h)
    assert abs(d_gpu / d_orc - 1) < 1e-2
    P.close()


@pytest.mark.parametrize("M", [1, 5, 40, 240])
def test_kerr_manakov(gpu_lib, M):
    """The paper's Eq. (1) nonlinear operator on the GPU vs the FP64 oracle."""
    mm = gpu_lib
    T = 512
    rng = np.random.default_rng((15, M))
    kappa = W.xpm_matrix(M, rng)
    beta = np.zeros((M, 1))
    P = mm.Propagator(M, T, 0.5, beta, None, 1.3, 0.05, 0.05, kappa=kappa)
    assert P.kerr_path == "manakov"
    X = crandn(rng, M, T)
    Y = host(P.kerr(dev(X)))
    ref = 0.05 * oracle.KerrManakov(kappa.astype(np.float64), 1.3)(X.astype(np.complex128))
    assert rel(Y, ref) < 2e-6
    P.close()


def test_manakov_propagation(gpu_lib):
    """Whole RK4IP propagation with the paper's Eq. (1) model (30 rows = 15 spatial modes
    x 2 polarizations, attenuation on) vs the oracle."""
    mm = gpu_lib
    p = W.manakov_problem(M=30, T=2 ** 12, n_steps=20)
    print(f"propagate manakov M={p.M} T={p.T} steps={p.n_steps}", flush=True)
    P = mm.Propagator.from_problem(p)
    assert P.kerr_path == "manakov"
    out, st = P.propagate(p.A0, stats=True)
    ref = oracle.propagate(p.A0, p.beta, p.alpha, None, p.gamma, p.dt, p.h, p.n_steps,
                           kerr=oracle.KerrManakov(p.kappa.astype(np.float64), p.gamma))
    err = rel(out, ref)
    print(f"  rel L2 = {err:.3e}", flush=True)
    assert err < 1e-5
    # attenuation: power decays as exp(-alpha L) exactly (the Kerr term conserves it)
    assert abs(st["power_out"] / st["power_in"] / np.exp(-p.alpha[0] * p.L) - 1) < 1e-5
    P.close()


@pytest.mark.parametrize("name,kw", [("qpsk6", dict(T=2 ** 12, n_steps=20)),
                                     ("wdm36", dict(T=2 ** 12, n_steps=10))])
def test_ssfm_rk4_propagation(gpu_lib, name, kw):
    """The paper's SSFM-RK4 variant (Eq. 4) through the same kernels vs the oracle."""
    mm = gpu_lib
    p = W.make_problem(name, **kw)
    P = mm.Propagator.from_problem(p, method=mm.SSFM_RK4)
    out = P.propagate(p.A0)
    kern = oracle.KerrGeneric(p.S, p.gamma)
    ref = oracle.propagate(p.A0, p.beta, None, p.S, p.gamma, p.dt, p.h, p.n_steps, kerr=kern,
                           method="ssfm_rk4")
    err = rel(out, ref)
    print(f"ssfm {name}: rel L2 = {err:.3e}", flush=True)
    assert err < 1e-5
    # device-resident advance equals the host-path propagation bit for bit
    import torch
    A = dev(p.A0)
    P.advance(A, p.n_steps)
    torch.cuda.synchronize()
    assert np.array_equal(host(A), out)
    P.close()


def test_ssfm_agrawal_manakov_propagation(gpu_lib):
    """The paper's SSFM-Agrawal variant (Eq. 4, iterated trapezoidal nonlinear
    step) with the Manakov operator of Eq. (1), 30 rows, attenuation on."""
    mm = gpu_lib
    p = W.manakov_problem(M=30, T=2 ** 12, n_steps=20)
    P = mm.Propagator.from_problem(p, method=mm.SSFM_AGRAWAL)
    out, st = P.propagate(p.A0, stats=True)
    ref = oracle.propagate(p.A0, p.beta, p.alpha, None, p.gamma, p.dt, p.h, p.n_steps,
                           kerr=oracle.KerrManakov(p.kappa.astype(np.float64), p.gamma), method="ssfm_agrawal")
    err = rel(out, ref)
    print(f"ssfm_agrawal manakov M={p.M} T={p.T}: rel L2 = {err:.3e}", flush=True)
    assert err < 1e-5
    # the nonlinear step is a pure phase: power decays exactly as exp(-alpha L)
    assert abs(st["power_out"] / st["power_in"] / np.exp(-p.alpha[0] * p.L) - 1) < 1e-5
    P.close()
    q = W.make_problem("qpsk6", T=2 ** 10, n_steps=1)
    with pytest.raises(mm.MMNLSEError):       # tensor plans have no phase form
        mm.Propagator.from_problem(q, method=mm.SSFM_AGRAWAL)


@pytest.mark.parametrize("name", ["manakov", "qpsk6"])
def test_amplified_spans(gpu_lib, name):
    """Spans with the loss-compensating amplifier after each (Section 5's
    two-span link), against the oracle; the device path span by span
    (advance, amplify) and a run with diagnostics every 4 steps give the same
    bits; with uniform attenuation the output power matches the oracle's."""
    import dataclasses
    import torch
    mm = gpu_lib
    if name == "manakov":
        p = W.manakov_problem(M=30, T=2 ** 12, n_steps=40)
        kerr = oracle.KerrManakov(p.kappa.astype(np.float64), p.gamma)
    else:
        p = dataclasses.replace(W.make_problem("qpsk6", T=2 ** 12, n_steps=20), alpha=np.full(6, 0.2))
        kerr = None
    k = 10
    span = k * p.h
    print(f"spans {name}: M={p.M} T={p.T} steps={p.n_steps} span={span:g} km", flush=True)
    P = mm.Propagator.from_problem(p, span=span)
    out, st = P.propagate(p.A0, stats=True)
    ref = oracle.propagate(p.A0, p.beta, p.alpha, p.S, p.gamma, p.dt, p.h, p.n_steps, kerr=kerr,
                           span_steps=k)
    err = rel(out, ref)
    print(f"  rel L2 = {err:.3e}, power out/in = {st['power_out'] / st['power_in']:.8f}", flush=True)
    assert err < 1e-5
    assert abs(st["power_out"] / oracle.power(ref, p.dt) - 1) < 1e-5
    A = dev(p.A0)
    for _ in range(p.n_steps // k):
        P.advance(A, k)
        P.amplify(A)
    torch.cuda.synchronize()
    assert np.array_equal(host(A), out)
    Q = mm.Propagator.from_problem(p, span=span, diag_every=4)
    out_d, st_d = Q.propagate(p.A0, stats=True)
    assert np.array_equal(out_d, out)
    assert st_d["diag_points"] == -(-p.n_steps // 4)
    Q.close()
    P.close()
    R = mm.Propagator.from_problem(p)
    with pytest.raises(mm.MMNLSEError):       # no spans configured
        R.amplify(dev(p.A0))
    R.close()


def test_method_accuracy_per_step(gpu_lib):
    """RK4IP against the two split-step variants of Section 3.1 on the Manakov
    model (30 rows, launch amplitude x6, 2 km), errors against an FP64 RK4IP
    run of 320 steps: at 20, 40 and 80 steps RK4IP is the most accurate and
    SSFM-Agrawal the least, and halving h from 40 to 80 steps divides the
    errors as fourth order (RK4IP; ratio 38 measured) and second order
    (the split steps; 7.7 and 4.1) predict."""
    mm = gpu_lib
    p = W.manakov_problem(M=30, T=2 ** 12, n_steps=20)
    A0 = (p.A0.astype(np.complex128) * 6.0).astype(np.complex64)
    L = 2.0
    kerr = oracle.KerrManakov(p.kappa.astype(np.float64), p.gamma)
    ref = oracle.propagate(A0, p.beta, p.alpha, None, p.gamma, p.dt, L / 320, 320, kerr=kerr)
    err = {}
    for name, m in (("rk4ip", mm.RK4IP), ("ssfm_rk4", mm.SSFM_RK4), ("ssfm_agrawal", mm.SSFM_AGRAWAL)):
        err[name] = []
        for n in (20, 40, 80):
            P = mm.Propagator(p.M, p.T, p.dt, p.beta, None, p.gamma, L / n, L, alpha=p.alpha,
                              kappa=p.kappa, method=m)
            err[name].append(rel(P.propagate(A0), ref))
            P.close()
        print(f"{name:13s} " + " ".join(f"{e:.3e}" for e in err[name]), flush=True)
    for i in range(3):
        assert err["rk4ip"][i] < err["ssfm_rk4"][i] < err["ssfm_agrawal"][i]
    ratio = {k: v[1] / v[2] for k, v in err.items()}
    assert ratio["rk4ip"] > 16
    assert 3 < ratio["ssfm_rk4"] < 12
    assert 3 < ratio["ssfm_agrawal"] < 6


def test_propagate_periodic_diagnostics(gpu_lib):
    """diag_every = 64 on a third-order soliton over one period (256 steps): four
    diagnostic points, a result bit-identical to the undiagnosed run, and the
    largest power drift and step-doubling estimate (delta/15) equal to the
    oracle's at the same four states.  At this coarse step both are scheme
    error (drift ~4e-4, delta up to ~8e-3), far above the FP32 rounding."""
    mm = gpu_lib
    p = W.soliton_problem(T=1024, noise=0.0)
    A0 = (3.0 * p.A0).astype(np.complex64)
    z0 = math.pi / 2 * p.meta["T0"] ** 2 / abs(p.beta[0, 2])
    n, every = 256, 64
    P = mm.Propagator(1, p.T, p.dt, p.beta, p.S, p.gamma, z0 / n, z0, diag_every=every)
    out, st = P.propagate(A0, stats=True)
    Q = mm.Propagator(1, p.T, p.dt, p.beta, p.S, p.gamma, z0 / n, z0)
    ref_gpu, st0 = Q.propagate(A0, stats=True)
    assert st["diag_points"] == n // every and st0["diag_points"] == 0
    assert np.array_equal(out, ref_gpu)
    A = A0.astype(np.complex128)
    p0 = oracle.power(A, p.dt)
    est, drift = [], []
    for _ in range(n // every):
        A = oracle.propagate(A, p.beta, None, p.S, p.gamma, p.dt, z0 / n, every)
        d, _ = oracle.step_doubling_estimate(A, p.beta, None, p.S, p.gamma, p.dt, z0 / n)
        est.append(d / 15.0)
        drift.append(abs(oracle.power(A, p.dt) / p0 - 1.0))
    print(f"power drift: GPU {st['power_drift_max']:.4e}, oracle {max(drift):.4e}; "
          f"local error estimate: GPU {st['local_err_max']:.4e}, oracle {max(est):.4e}", flush=True)
    assert st["power_drift_max"] == pytest.approx(max(drift), rel=0.02)
    assert st["local_err_max"] == pytest.approx(max(est), rel=0.05)
    P.close()
    Q.close()
    with pytest.raises(mm.MMNLSEError):
        mm.Propagator(1, p.T, p.dt, p.beta, p.S, p.gamma, z0 / n, z0, diag_every=-1)
