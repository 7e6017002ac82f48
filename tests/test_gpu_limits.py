"""Edge and maximum sizes of the boundary, against the oracle or closed forms.

  * the largest transforms (T = 2^18 .. 2^20: four-step with 512- and
    1024-point passes);
  * the matrix-core contraction in its two widest workgroup shapes, M = 126
    (two row groups) and M = 256 (the largest M, one row group), with a
    tensor that is a sum of K symmetric rank-1 terms,
        S = sum_k c_k u_k (x) u_k (x) u_k (x) u_k,
    for which N_p = i gamma sum_k c_k u_kp (u_k . X)^2 conj(u_k . X) in closed
    form (the oracle's rank-1 pin), so no M^4 reference sum is needed;
  * rows too short for the 128-sample workgroup (T = 64);
  * zero steps.

Tolerance of the wide contractions: the packed GEMM accumulates P = M(M+1)/2
products per output in FP32, two per matrix-core step, so rounding grows like
sqrt(P/2) * 6e-8: 3.8e-6 at M = 126 and 7.7e-6 at M = 256; the bars are about
three times that.
"""

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


def crandn(rng, *shape):
    return ((rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2)).astype(np.complex64)


@pytest.mark.parametrize("T", [2 ** 18, 2 ** 19, 2 ** 20])
def test_linear_half_step_largest_T(gpu_lib, T):
    mm = gpu_lib
    import torch
    M, dt = 2, 0.05
    print(f"linear_half_step T={T}", flush=True)
    rng = np.random.default_rng((23, T))
    beta = np.column_stack([rng.uniform(-50, 50, M), rng.uniform(-20, 20, M), rng.uniform(-25, -15, M)])
    S = W.symmetric_gaussian_tensor(M, rng).astype(np.float32)
    P = mm.Propagator(M, T, dt, beta, S, 1.0, 0.1, 0.1)
    X = crandn(rng, M, T)
    Y = P.linear_half_step(torch.from_numpy(X).cuda()).cpu().numpy()
    E = oracle.half_step_propagator(oracle.angular_frequencies(T, dt), beta, None, 0.1)
    ref = oracle.apply_linear(X.astype(np.complex128), E)
    err = rel(Y, ref)
    print(f"  rel L2 = {err:.3e}", flush=True)
    assert err < 1e-6
    P.close()


def _rank_k_tensor(M, rng, K=3):
    """S_plmn = sum_k c_k a_k(p) b_k(l) b_k(m) a_k(n) with a_k != b_k: symmetric
    in (l, m) and in (p, n), as the packed contraction needs, but not under
    p <-> l, so that a transposed index changes the result.  Its Kerr term has
    the closed form  i gamma sum_k c_k a_k(p) (b_k . X)^2 conj(a_k . X)."""
    a = rng.standard_normal((K, M)).astype(np.float32)
    b = rng.standard_normal((K, M)).astype(np.float32)
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    c = rng.uniform(0.5, 1.5, K).astype(np.float32)
    S = np.zeros((M,) * 4, dtype=np.float32)
    for k in range(K):
        pn = c[k] * (a[k][:, None] * a[k][None, :])   # exactly symmetric products
        lm = b[k][:, None] * b[k][None, :]
        for p in range(M):   # one p-slab at a time keeps the temporaries at M^3
            S[p] += lm[:, :, None] * pn[p][None, None, :]
    return S, a.astype(np.float64), b.astype(np.float64), c.astype(np.float64)


@pytest.mark.parametrize("M,tol", [(126, 1.2e-5), (256, 2.5e-5)])
def test_kerr_mfma_widest_shapes(gpu_lib, M, tol):
    mm = gpu_lib
    import torch
    T, gamma, h = 256, 1.3, 0.05
    print(f"kerr mfma M={M}: building the tensor", flush=True)
    rng = np.random.default_rng((29, M))
    S, a, b, c = _rank_k_tensor(M, rng)
    beta = np.zeros((M, 1))
    P = mm.Propagator(M, T, 0.5, beta, S, gamma, h, h, symmetric=True)
    del S
    assert P.kerr_path == "mfma"
    X = crandn(rng, M, T)
    Y = P.kerr(torch.from_numpy(X).cuda()).cpu().numpy()
    Xd = X.astype(np.complex128)
    ya, yb = a @ Xd, b @ Xd                            # [K, T]: a_k . X, b_k . X
    ref = 1j * gamma * h * np.einsum("k,kp,kt->pt", c, a, yb * yb * np.conj(ya))
    err = rel(Y, ref)
    worst = float(np.max(np.linalg.norm(Y - ref, axis=1) / np.linalg.norm(ref, axis=1)))
    print(f"  rel L2 = {err:.3e}, worst mode {worst:.3e}", flush=True)
    assert err < tol
    assert worst < 4 * tol
    P.close()


def test_kerr_mfma_short_rows(gpu_lib):
    """T = 64 is below the 128-sample workgroup: the 32-sample shape runs."""
    mm = gpu_lib
    import torch
    M, T = 6, 64
    rng = np.random.default_rng(31)
    S = W.symmetric_gaussian_tensor(M, rng).astype(np.float32)
    P = mm.Propagator(M, T, 0.5, np.zeros((M, 1)), S, 1.3, 0.05, 0.05)
    assert P.kerr_path == "mfma"
    X = crandn(rng, M, T)
    Y = P.kerr(torch.from_numpy(X).cuda()).cpu().numpy()
    ref = 0.05 * oracle.kerr_term(X.astype(np.complex128), S.astype(np.float64), 1.3)
    assert rel(Y, ref) < 2e-6
    P.close()


def test_zero_steps_leave_the_field_unchanged(gpu_lib):
    mm = gpu_lib
    import torch
    p = W.make_problem("qpsk6", T=2 ** 12, n_steps=1)
    P = mm.Propagator.from_problem(p)
    A = torch.from_numpy(p.A0).cuda()
    P.advance(A, 0)
    torch.cuda.synchronize()
    assert np.array_equal(A.cpu().numpy(), p.A0)
    with pytest.raises(mm.MMNLSEError):
        P.advance(A, -1)
    P.close()


@pytest.mark.parametrize("name,kw", [("qpsk6", dict(T=2 ** 10, n_steps=1)), ("wdm36", dict(T=2 ** 10, n_steps=1))])
def test_kerr_work_counts(gpu_lib, name, kw):
    """The matrix-core path reports the packed entries it multiplies: all P^2
    for a dense tensor; for the mode-group-masked wdm36 tensor the nonzero
    count of the packed matrix Sp[(p,n)][(l,m)] = w S[p,l,m,n], and at least
    that many multiplied."""
    mm = gpu_lib
    p = W.make_problem(name, **kw)
    P = mm.Propagator.from_problem(p)
    work = P.kerr_work()
    M = p.M
    pairs = [(i, j) for i in range(M) for j in range(i, M)]
    a = np.array([x[0] for x in pairs])
    b = np.array([x[1] for x in pairs])
    Sp = p.S[a[:, None], a[None, :], b[None, :], b[:, None]]
    nnz = int(np.count_nonzero(Sp))
    print(f"{name}: dense {work['dense']:.0f}, multiplied {work['multiplied']:.0f}, nonzero {work['nonzero']:.0f}",
          flush=True)
    assert work["dense"] == len(pairs) ** 2
    assert work["nonzero"] == nnz
    plan = mm.kerr_plan(p.S, mm.FP32)
    assert nnz <= work["multiplied"] <= 32 * plan["nrt"] * plan["Ppad"]
    # the per-pass kernel multiplies its passes' listed blocks (the host plan's
    # count); the group kernel only the nonzero (row tile, k-step) blocks
    assert work["multiplied"] <= plan["entries"]["multiplied"]
    P.close()


def test_misaligned_device_field_is_rejected(gpu_lib):
    """The transforms move two samples per 16-byte access: a field pointer
    that is only 8-byte aligned is refused before any launch, and the plan
    keeps working with an aligned one."""
    mm = gpu_lib
    import torch
    p = W.make_problem("qpsk6", T=2 ** 10, n_steps=2)
    P = mm.Propagator.from_problem(p)
    flat = torch.zeros(p.M * p.T + 1, dtype=torch.complex64, device="cuda")
    A_bad = flat[1:]
    assert A_bad.data_ptr() % 16 == 8
    for call in (lambda: P.advance(A_bad, 1), lambda: P.linear_half_step(A_bad)):
        with pytest.raises(mm.MMNLSEError) as e:
            call()
        assert e.value.status == 1
    A = torch.from_numpy(p.A0).cuda()
    P.advance(A, p.n_steps)
    torch.cuda.synchronize()
    assert np.array_equal(A.cpu().numpy(), P.propagate(p.A0))
    P.close()
