"""Plain FP64 reference of one RK4IP step of the coupled multimode NLSE.

TEST INFRASTRUCTURE ONLY (see the package docstring): used by tests, the
smoke check and the benchmark's CPU baseline; never by the library.

What it computes, following Brehler et al., "Simulation of Nonlinear Signal
Propagation in Multimode Fibers on Multi-GPU Systems" (CPC):

* the linear operator of Eq. (1): attenuation plus the Taylor series of the
  propagation constant, applied in the frequency domain (Section 3.1);
* the Kerr term in the general tensor form N_p = i*gamma*sum_{l,m,n}
  S_plmn A_l A_m conj(A_n) of the multimode NLSE the paper cites in Section 2
  (for one mode it is the paper's gamma*|A|^2*A);
* the RK4IP step of Eq. (6a-f) with separation distance z' = z + h/2
  (Section 3.2, Eq. 5).

Readings of the paper taken here (each is also a test below):

* Eq. (6b) prints its brackets garbled; k1 is read as the half-step linear
  propagator applied to h*N(A(z)), as Eq. (5) with z' = z+h/2 implies.
* Fourier convention: numpy's forward kernel exp(-i w t).  The time-domain
  operator i * (i^n/n!) beta_n d^n/dt^n then becomes i beta_n (-w)^n / n! per
  angular frequency w, the Nyquist bin taking numpy's negative frequency.
* A_out[p] is the output index of S, the last index n is the conjugated one.

Pins (tests/test_oracle_pins.py, all CPU):

* linear operator vs analytic derivatives of a Gaussian (every beta_n sign);
* beta1 shift by an integer number of samples equals a circular roll;
* beta2 broadening of a Gaussian vs the textbook closed form;
* single-entry S tensors and linearity in S (index wiring, conjugated index);
* power conservation exactly for the pair-exchange symmetry S_plmn = S_lpnm;
* rank-1 S = u x u x u x u closed-form solution;
* self-phase modulation exp(i gamma |A|^2 z) and CW + beta0 phase (IP frame);
* classical RK4 reduction when the linear operator vanishes;
* fundamental soliton and 4th-order convergence under step halving;
* packed symmetric Kerr == generic Kerr for symmetric S;
* Manakov/XPM form of Eq. (1): exact per-mode phase rotation without
  dispersion, and equality with the tensor form S_plmn = kappa_pm d_lp d_mn;
* SSFM-RK4 (Eq. 4): exact for the linear part, identical to RK4IP without
  dispersion, second order on the soliton;
* SSFM-Agrawal (Eq. 4, iterated trapezoidal nonlinear step, Manakov form):
  exact for the linear part, exact without dispersion for any h, second
  order on the soliton (first order with a single pass);
* spans with loss-compensating amplifiers: lossless Gaussian GVD at the
  span ends and exp(-alpha z/2) between them; lossy SPM converging at fourth
  order to its closed form with the effective length (1 - e^{-alpha z})/alpha;
* adaptive step size (step doubling): exact and doubling steps for the
  linear part, accepted steps scaling as tol^(-1/5) (fifth-order local
  error, Section 3.2), global error below the summed local tolerances,
  recovery from an oversized first step.

Units: t in ps, z in km, power in W, w in rad/ps, beta_n in ps^n/km.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "time_grid", "angular_frequencies", "linear_operator", "half_step_propagator",
    "apply_linear", "KerrGeneric", "KerrPacked", "KerrManakov", "kerr_term", "rk4ip_step",
    "propagate", "power", "step_doubling_estimate", "ssfm_rk4_step", "ssfm_agrawal_step", "propagate_adaptive",
    "propagate_steps", "StepControlError", "amplifier_gain",
]


# ----------------------------------------------------------------------------
# grids and the linear part (Eq. 1, operator L)
# ----------------------------------------------------------------------------

def time_grid(T: int, dt: float) -> np.ndarray:
    """Sample times t_j = (j - T/2) dt."""
    return (np.arange(T) - T // 2) * dt


def angular_frequencies(T: int, dt: float) -> np.ndarray:
    """w_k = 2 pi fftfreq(T, dt)[k] in rad/ps (numpy bin order)."""
    return 2.0 * np.pi * np.fft.fftfreq(T, dt)


def linear_operator(omega: np.ndarray, beta: np.ndarray, alpha: np.ndarray | None) -> np.ndarray:
    """L(w) per mode, Eq. (1): -alpha/2 + i sum_n beta_n (-w)^n / n!.

    With the forward kernel exp(-i w t), d/dt acts as multiplication by i w,
    so the time-domain term i (i^n / n!) beta_n d^n/dt^n becomes
    i (i * i w)^n beta_n / n! = i beta_n (-w)^n / n!.
    ``beta`` is [M, n_beta]; returns [M, T] complex128.
    """
    beta = np.atleast_2d(np.asarray(beta, dtype=np.float64))
    M, nb = beta.shape
    L = np.zeros((M, omega.size), dtype=np.complex128)
    for n in range(nb):
        L += 1j * beta[:, n:n + 1] * (-omega[None, :]) ** n / math.factorial(n)
    if alpha is not None:
        L -= 0.5 * np.asarray(alpha, dtype=np.float64)[:, None]
    return L


def half_step_propagator(omega: np.ndarray, beta: np.ndarray, alpha: np.ndarray | None,
                         h: float) -> np.ndarray:
    """exp(h/2 * L(w)) per mode and frequency bin, [M, T] complex128."""
    return np.exp(0.5 * h * linear_operator(omega, beta, alpha))


def apply_linear(X: np.ndarray, E: np.ndarray) -> np.ndarray:
    """Apply a frequency-domain factor E to every row: ifft(E * fft(X))."""
    return np.fft.ifft(E * np.fft.fft(X, axis=-1), axis=-1)


# ----------------------------------------------------------------------------
# the Kerr term N(X)_p = i gamma sum_{l,m,n} S_plmn X_l X_m conj(X_n)
# ----------------------------------------------------------------------------

class KerrGeneric:
    """Kerr term for any real S (no symmetry assumed).

    C_pn(t) = sum_{l,m} S_plmn X_l(t) X_m(t) is one matrix product of the
    [(p,n), (l,m)] view of S with the [(l,m), t] products; then
    N_p(t) = i gamma sum_n C_pn(t) conj(X_n(t)).  Chunked over t only to bound
    memory.
    """

    def __init__(self, S: np.ndarray, gamma: float, chunk: int = 4096):
        S = np.asarray(S, dtype=np.float64)
        M = S.shape[0]
        if S.shape != (M, M, M, M):
            raise ValueError("S must be [M,M,M,M]")
        self.M = M
        self.gamma = float(gamma)
        self.chunk = chunk
        # rows (p, n), columns (l, m)
        self.Smat = np.ascontiguousarray(S.transpose(0, 3, 1, 2).reshape(M * M, M * M))

    def __call__(self, X: np.ndarray) -> np.ndarray:
        M = self.M
        X = np.asarray(X, dtype=np.complex128)
        T = X.shape[1]
        out = np.empty((M, T), dtype=np.complex128)
        for s in range(0, T, self.chunk):
            x = X[:, s:s + self.chunk]
            B = (x[:, None, :] * x[None, :, :]).reshape(M * M, -1)      # [(l,m), t]
            Br, Bi = np.ascontiguousarray(B.real), np.ascontiguousarray(B.imag)
            C = (self.Smat @ Br + 1j * (self.Smat @ Bi)).reshape(M, M, -1)  # [p, n, t]
            out[:, s:s + self.chunk] = 1j * self.gamma * np.einsum("pnt,nt->pt", C, np.conj(x))
        return out


class KerrPacked:
    """Kerr term for S symmetric in (l,m) and in (p,n).

    With q = (l <= m) and weight w_q = 2 for l < m (1 for l == m),
    C_pn = sum_q w_q S_p,l_q,m_q,n X_l X_m, and C_pn = C_np, so only the
    P = M(M+1)/2 rows p <= n are formed:
    N_p = i gamma (sum_{n >= p} C_pn conj(X_n) + sum_{n < p} C_np conj(X_n)).
    """

    def __init__(self, S: np.ndarray, gamma: float, chunk: int = 4096):
        S = np.asarray(S, dtype=np.float64)
        M = S.shape[0]
        a, b = np.triu_indices(M)
        w = np.where(a < b, 2.0, 1.0)
        # rows r = (p=a_r, n=b_r), columns q = (l=a_q, m=b_q)
        self.Smat = np.ascontiguousarray(S[a[:, None], a[None, :], b[None, :], b[:, None]] * w[None, :])
        self.a, self.b = a, b
        self.off = a < b
        self.M = M
        self.gamma = float(gamma)
        self.chunk = chunk

    def __call__(self, X: np.ndarray) -> np.ndarray:
        X = np.asarray(X, dtype=np.complex128)
        a, b = self.a, self.b
        out = np.zeros_like(X)
        for s in range(0, X.shape[1], self.chunk):
            x = X[:, s:s + self.chunk]
            B = x[a] * x[b]                                            # [q, t]
            Br, Bi = np.ascontiguousarray(B.real), np.ascontiguousarray(B.imag)
            C = self.Smat @ Br + 1j * (self.Smat @ Bi)                  # [r, t]
            o = np.zeros_like(x)
            np.add.at(o, a, C * np.conj(x[b]))
            np.add.at(o, b[self.off], C[self.off] * np.conj(x[a[self.off]]))
            out[:, s:s + self.chunk] = 1j * self.gamma * o
        return out


class KerrManakov:
    """The paper's own nonlinear operator, Eq. (1):
    N_a = i gamma (kappa_aa |X_a|^2 + sum_{b != a} kappa_ab |X_b|^2) X_a
        = i gamma (sum_b kappa_ab |X_b|^2) X_a,
    with a real coupling matrix kappa (rows = modes incl. polarizations)."""

    def __init__(self, kappa: np.ndarray, gamma: float):
        self.kappa = np.asarray(kappa, dtype=np.float64)
        if self.kappa.ndim != 2 or self.kappa.shape[0] != self.kappa.shape[1]:
            raise ValueError("kappa must be [M,M]")
        self.gamma = float(gamma)

    def __call__(self, X: np.ndarray) -> np.ndarray:
        X = np.asarray(X, dtype=np.complex128)
        phase = self.kappa @ (np.abs(X) ** 2)        # [a, t]
        return 1j * self.gamma * phase * X


def kerr_term(X: np.ndarray, S: np.ndarray, gamma: float) -> np.ndarray:
    """N(X) for any S (generic form)."""
    return KerrGeneric(S, gamma)(X)


# ----------------------------------------------------------------------------
# the RK4IP step, Eq. (6a-f)
# ----------------------------------------------------------------------------

def rk4ip_step(A: np.ndarray, E: np.ndarray, h: float, N) -> np.ndarray:
    """Advance A(z) to A(z+h); E = exp(h/2 L), N = callable Kerr term."""
    AI = apply_linear(A, E)                                   # (6a)
    k1 = apply_linear(h * N(A), E)                            # (6b)
    k2 = h * N(AI + k1 / 2.0)                                 # (6c)
    k3 = h * N(AI + k2 / 2.0)                                 # (6d)
    k4 = h * N(apply_linear(AI + k3, E))                      # (6e)
    return apply_linear(AI + k1 / 6.0 + k2 / 3.0 + k3 / 3.0, E) + k4 / 6.0   # (6f)


def ssfm_rk4_step(A: np.ndarray, E: np.ndarray, h: float, N) -> np.ndarray:
    """Symmetric split-step of Eq. (4): a half linear step, the nonlinear part
    over h (A' = N(A), classical fourth-order Runge-Kutta: the paper's
    SSFM-RK4 variant), another half linear step.  Global error O(h^2)."""
    X = apply_linear(A, E)
    k1 = h * N(X)
    k2 = h * N(X + k1 / 2.0)
    k3 = h * N(X + k2 / 2.0)
    k4 = h * N(X + k3)
    X = X + (k1 + 2.0 * k2 + 2.0 * k3 + k4) / 6.0
    return apply_linear(X, E)


def ssfm_agrawal_step(A: np.ndarray, E: np.ndarray, h: float, N, iterations: int = 2) -> np.ndarray:
    """Symmetric split-step of Eq. (4) with the nonlinear integral taken by the
    iterated trapezoidal rule (the paper's "SSFM-Agrawal", after Agrawal's
    Nonlinear Fiber Optics), for the Manakov/XPM operator of Eq. (1).  That
    operator multiplies each mode by i gamma Phi_a, Phi = kappa |A|^2, so its
    exponential is a phase rotation: exp(int N dz) A_a = exp(i gamma int Phi_a dz) A_a.
    int_z^{z+h} Phi dz ~ h/2 (Phi(z) + Phi(z+h)); Phi(z+h) is first taken equal
    to Phi(z), then recomputed from the field reached at z+h, `iterations`
    passes in all.  N must be a KerrManakov.  Global error O(h^2)."""
    kappa, gamma = N.kappa, N.gamma
    phi_z = kappa @ (np.abs(A) ** 2)
    Ah = apply_linear(A, E)
    phi_end = phi_z
    for _ in range(iterations):
        out = apply_linear(Ah * np.exp(0.5j * gamma * h * (phi_z + phi_end)), E)
        phi_end = kappa @ (np.abs(out) ** 2)
    return out


def _kerr_for(S, gamma, kerr):
    if kerr is not None and not isinstance(kerr, str):
        return kerr
    S = np.asarray(S)
    if kerr == "packed":
        return KerrPacked(S, gamma)
    return KerrGeneric(S, gamma)


def propagate(A0: np.ndarray, beta: np.ndarray, alpha: np.ndarray | None, S: np.ndarray,
              gamma: float, dt: float, h: float, n_steps: int, kerr=None,
              callback=None, method: str = "rk4ip", span_steps: int = 0) -> np.ndarray:
    """n_steps fixed steps of size h from A0 (promoted to complex128).

    ``method`` is "rk4ip" (Eq. 6, default), "ssfm_rk4" (Eq. 4 with an RK4
    nonlinear step) or "ssfm_agrawal" (Eq. 4 with the iterated trapezoidal
    nonlinear step; Manakov operator only).  ``kerr`` may be None/"generic", "packed" (S must be
    symmetric in (l,m) and (p,n)), or a ready callable.  ``callback(step, A)``
    is called after each step when given.

    ``span_steps`` = k > 0 puts an amplifier after every k steps (a span of
    k*h km): see ``amplifier_gain``; the callback sees the amplified field.
    """
    A = np.array(A0, dtype=np.complex128, copy=True)
    M, T = A.shape
    E = half_step_propagator(angular_frequencies(T, dt), beta, alpha, h)
    N = _kerr_for(S, gamma, kerr)
    if method == "rk4ip":
        step = rk4ip_step
    elif method == "ssfm_rk4":
        step = ssfm_rk4_step
    elif method == "ssfm_agrawal":
        if not isinstance(N, KerrManakov):
            raise ValueError("ssfm_agrawal needs the Manakov operator (kerr=KerrManakov(kappa, gamma))")
        step = ssfm_agrawal_step
    else:
        raise ValueError(method)
    if span_steps < 0:
        raise ValueError("span_steps < 0")
    g = amplifier_gain(alpha, M, span_steps * h) if span_steps else None
    for s in range(n_steps):
        A = step(A, E, h, N)
        if g is not None and (s + 1) % span_steps == 0:
            A = g[:, None] * A
        if callback is not None:
            callback(s + 1, A)
    return A


def amplifier_gain(alpha: np.ndarray | None, M: int, span: float) -> np.ndarray:
    """Field gain per mode of the noiseless, flat-gain amplifier placed after
    each fiber span (Section 5: two 80 km spans, the fiber loss compensated
    after each).  Flat in frequency; it restores the span's power loss
    exp(-alpha_p span) of each mode, so the field gain is exp(alpha_p span / 2)."""
    a = np.zeros(M) if alpha is None else np.asarray(alpha, dtype=np.float64)
    return np.exp(0.5 * a * span)


def power(A: np.ndarray, dt: float) -> float:
    """Total power integral dt * sum_p sum_t |A_p(t)|^2 (W ps)."""
    return float(dt * np.sum(np.abs(np.asarray(A, dtype=np.complex128)) ** 2))


def step_doubling_estimate(A: np.ndarray, beta, alpha, S, gamma: float, dt: float, h: float,
                           kerr=None) -> tuple[float, np.ndarray]:
    """Richardson estimate for the local error of two h-steps from A.

    delta = ||fine - coarse|| / ||fine|| with fine = two steps of h and
    coarse = one step of 2h from the same state; for a 4th-order scheme the
    error of ``fine`` is about delta/15.  Returns (delta, fine).
    """
    M, T = np.shape(A)
    w = angular_frequencies(T, dt)
    N = _kerr_for(S, gamma, kerr)
    A = np.asarray(A, dtype=np.complex128)
    Eh = half_step_propagator(w, beta, alpha, h)
    E2h = half_step_propagator(w, beta, alpha, 2.0 * h)
    fine = rk4ip_step(rk4ip_step(A, Eh, h, N), Eh, h, N)
    coarse = rk4ip_step(A, E2h, 2.0 * h, N)
    nf, nd = np.linalg.norm(fine), np.linalg.norm(fine - coarse)
    delta = float(nd / nf) if nf > 0 else (0.0 if nd == 0 else math.nan)   # 0 for a zero field
    return delta, fine


# ----------------------------------------------------------------------------
# adaptive step size from the step-doubling estimate
# ----------------------------------------------------------------------------
#
# The paper integrates with fixed steps.  The controller below is the textbook
# step-doubling scheme for Runge-Kutta methods (Press et al., Numerical
# Recipes, "Adaptive Stepsize Control for Runge-Kutta"), with the exponent
# fixed by the order the paper states for RK4IP (Section 3.2: local error of
# fifth order, so delta ~ h^5):
#
#   trial h from z:   coarse = one step of h,  fine = two steps of h/2,
#                     delta  = ||fine - coarse|| / ||fine||
#   accept iff delta <= tol: the state becomes `fine` and z advances by h;
#   next trial:       h <- min(h_max, h * clamp(0.9 (tol/delta)^(1/5), 0.5, 2))
#                     (factor 2 when delta == 0, 0.5 when delta is not finite),
#                     cut to the distance left.

LENGTH_EPS = 1e-12  # propagation ends when less than this fraction of the length is left


class StepControlError(RuntimeError):
    """The controller asked for a step below h_min or ran out of trials."""


def step_factor(delta: float, tol: float) -> float:
    """Next-trial step factor; a non-finite delta (a trial that overflowed) is
    a rejection with the largest cut."""
    if not math.isfinite(delta):
        return 0.5
    if delta == 0.0:
        return 2.0
    return min(2.0, max(0.5, 0.9 * (tol / delta) ** 0.2))


def propagate_adaptive(A0: np.ndarray, beta: np.ndarray, alpha: np.ndarray | None, S, gamma: float,
                       dt: float, length: float, tol: float, h_init: float, h_min: float = 0.0,
                       h_max: float = math.inf, max_trials: int = 100000, kerr=None):
    """Propagate over `length` with step-doubling control (see above).

    Returns (A, trials) with one (z, h, delta, accepted) tuple per trial.
    Raises StepControlError when the next step would fall below h_min or
    max_trials trials did not reach the end.
    """
    A = np.array(A0, dtype=np.complex128, copy=True)
    N = _kerr_for(S, gamma, kerr)
    z, h, trials = 0.0, min(h_init, h_max), []
    while length - z > LENGTH_EPS * length:
        if h < h_min:
            raise StepControlError(f"step {h} below h_min at z = {z}")
        if len(trials) >= max_trials:
            raise StepControlError(f"{max_trials} trials reached z = {z}")
        h = min(h, length - z)
        with np.errstate(over="ignore", invalid="ignore"):
            delta, fine = step_doubling_estimate(A, beta, alpha, S, gamma, dt, 0.5 * h, kerr=N)
        ok = delta <= tol   # False for NaN
        trials.append((z, h, delta, ok))
        if ok:
            A = fine
            z += h
        h = min(h_max, h * step_factor(delta, tol))
    return A, trials


def propagate_steps(A0: np.ndarray, beta: np.ndarray, alpha: np.ndarray | None, S, gamma: float,
                    dt: float, hs, kerr=None) -> np.ndarray:
    """RK4IP steps of the given sizes, in order (each with its own exp(h/2 L))."""
    A = np.array(A0, dtype=np.complex128, copy=True)
    w = angular_frequencies(A.shape[1], dt)
    N = _kerr_for(S, gamma, kerr)
    for h in hs:
        A = rk4ip_step(A, half_step_propagator(w, beta, alpha, h), h, N)
    return A
