"""Seeded synthetic launch fields, fiber coefficients and Kerr tensors.

Units throughout: time in ps, distance in km, power in W, frequency in THz
(1/ps), beta_n in ps^n/km, gamma in 1/(W km).

Every array is drawn from ``numpy.random.default_rng((190101895, cfg, stream,
sub))`` so that the FP64 reference and the GPU library see identical bytes.
Field and tensor dtypes are the stored ones (complex64 fields, FP32 tensor);
the one exception is the scalar soliton case, whose field is complex128.

Workloads (the shapes of the paper's multimode links, Sections 4-6 and
Tables 1-3; there is no public dataset behind them):

``soliton``  one mode, T=4096 over a 100 ps window, fundamental sech soliton
             (T0=2 ps, P0=|beta2|/(gamma T0^2)) plus 1e-6 relative complex
             Gaussian noise; beta2=-20 ps^2/km, gamma=1.3, L=1 km, h=5 m.
``qpsk6``    6 modes, T=2^14, 8 samples/symbol at 32 GBd, single-channel QPSK
             with raised-cosine spectrum (roll-off 0.1), 0 dBm per mode;
             beta0 ~ U(-1000,1000) rad/km, beta1 ~ U(-500,500) ps/km,
             beta2 ~ U(-25,-15) ps^2/km; dense symmetrised S; gamma=1,
             L=10 km, h=100 m.
``wdm36``    36 modes, T=2^16, 32 samples/symbol, 8 WDM channels on a 50 GHz
             grid, 16-QAM at 32 GBd, -2 dBm per channel; beta as ``qpsk6``;
             S as ``qpsk6`` with a mode-group mask zeroing >=70% of entries;
             gamma=1, L=50 km, h=50 m.
``wdm120``   120 modes, T=2^17, 16 samples/symbol, 4 channels, QPSK,
             -3 dBm per channel; beta1/beta2 from the paper's Table 3 per mode
             group; dense symmetrised S; gamma=0.5, L=10 km, h=20 m.
"""

from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

SEED_ROOT = 190101895

# independent random streams per workload
STREAM_S, STREAM_BETA, STREAM_SYMBOLS, STREAM_NOISE, STREAM_ARRIVALS, STREAM_MASK, \
    STREAM_REQUEST = range(7)

CONFIG_NAMES = ("soliton", "qpsk6", "wdm36", "serving", "wdm120")

# Table 3 of the paper: differential group delay per mode group (ps/km) and the
# group-averaged second-order dispersion (ps^2/km), mode groups 1..15.
_TABLE3_DBETA1 = (0.0, -7.32, -7.38, -7.48, -7.54, -7.60, -7.70, -7.79, -7.85,
                  -7.95, -8.04, -8.18, -8.23, -8.39, -8.61)
_TABLE3_BETA2 = (-23.1, -23.3, -23.5, -23.8, -24.0, -24.2, -24.5, -24.8, -25.0,
                 -25.3, -25.6, -25.9, -26.2, -26.7, -27.4)

BAUD_THZ = 0.032  # 32 GBd


def _rng(cfg: int, stream: int, sub: int = 0) -> np.random.Generator:
    return np.random.default_rng((SEED_ROOT, cfg, stream, sub))


@dataclass
class Problem:
    """One propagation problem: launch field plus everything the step needs."""

    name: str
    A0: np.ndarray            # [M, T] complex (row = mode, samples contiguous)
    beta: np.ndarray          # [M, n_beta] float64, beta_n in ps^n/km
    alpha: np.ndarray         # [M] float64, power attenuation 1/km
    S: np.ndarray             # [M, M, M, M] float32, index order (p, l, m, n)
    gamma: float              # 1/(W km)
    dt: float                 # ps
    h: float                  # km
    n_steps: int
    symmetric: bool           # S invariant under every index permutation
    meta: dict = field(default_factory=dict)
    kappa: np.ndarray | None = None   # [M, M] float32: Manakov / XPM form (S unused)

    @property
    def M(self) -> int:
        return self.A0.shape[0]

    @property
    def T(self) -> int:
        return self.A0.shape[1]

    @property
    def L(self) -> float:
        return self.h * self.n_steps


# ----------------------------------------------------------------------------
# mode groups (Table 2: group g holds g spatial modes, cumulative 1,3,6,...)
# ----------------------------------------------------------------------------

def mode_groups(M: int) -> np.ndarray:
    """Group index (0-based) of each of M modes, filling groups 1,2,3,... in order."""
    g = np.empty(M, dtype=np.int64)
    i, grp = 0, 0
    while i < M:
        n = min(grp + 1, M - i)
        g[i:i + n] = grp
        i += n
        grp += 1
    return g


def table3_beta(M: int) -> np.ndarray:
    """[M, 3] beta0/beta1/beta2 per mode from the paper's Table 3 (beta0 = 0)."""
    g = mode_groups(M)
    if g.max() >= len(_TABLE3_DBETA1):
        raise ValueError("Table 3 covers 15 mode groups (120 modes)")
    beta = np.zeros((M, 3))
    beta[:, 1] = np.asarray(_TABLE3_DBETA1)[g]
    beta[:, 2] = np.asarray(_TABLE3_BETA2)[g]
    return beta


# ----------------------------------------------------------------------------
# Kerr coupling tensors
# ----------------------------------------------------------------------------

def symmetric_gaussian_tensor(M: int, rng: np.random.Generator) -> np.ndarray:
    """Average of the 24 axis permutations of an iid N(0,1) tensor (float64)."""
    G = rng.standard_normal((M, M, M, M))
    acc = np.zeros_like(G)
    for perm in itertools.permutations(range(4)):
        np.add(acc, G.transpose(perm), out=acc)
    acc /= 24.0
    return acc


def pair_exchange_tensor(M: int, rng: np.random.Generator) -> np.ndarray:
    """Random real tensor with only the symmetry S[p,l,m,n] == S[l,p,n,m].

    Used by tests: it is the weakest symmetry under which the Kerr term
    conserves total power, and it is neither symmetric in (l,m) nor in (p,n).
    """
    G = rng.standard_normal((M, M, M, M))
    return 0.5 * (G + G.transpose(1, 0, 3, 2))


def mode_group_mask(M: int, frac: float, rng: np.random.Generator) -> tuple[np.ndarray, float]:
    """Permutation-invariant mask that zeroes whole mode-group classes.

    Each entry (p,l,m,n) belongs to the class of its sorted group quadruple.
    Classes other than the pure ones (g,g,g,g) are shuffled and zeroed in that
    order until at least ``frac`` of all entries are zero.  Returns the keep
    mask and the realised zero fraction.
    """
    g = mode_groups(M)
    G = int(g.max()) + 1
    idx = np.stack(np.meshgrid(g, g, g, g, indexing="ij"), axis=0)
    idx.sort(axis=0)
    code = ((idx[0] * G + idx[1]) * G + idx[2]) * G + idx[3]
    classes, counts = np.unique(code, return_counts=True)
    d = classes % G
    c = (classes // G) % G
    b = (classes // G // G) % G
    a = classes // G // G // G
    pure = (a == b) & (b == c) & (c == d)
    order = rng.permutation(np.nonzero(~pure)[0])
    total = M ** 4
    zeroed = 0
    drop = []
    for k in order:
        if zeroed >= frac * total:
            break
        drop.append(classes[k])
        zeroed += counts[k]
    keep = ~np.isin(code, np.asarray(drop, dtype=code.dtype))
    return keep, zeroed / total


def coupling_tensor(M: int, cfg: int, mask_frac: float = 0.0) -> tuple[np.ndarray, dict]:
    """Symmetrised Gaussian tensor, diagonal S[p,p,p,p] += 2, optional mask,
    normalised to max |S| = 1, rounded to FP32.  M = 1 gives S = [1]."""
    if M == 1:
        return np.ones((1, 1, 1, 1), dtype=np.float32), {"zero_fraction": 0.0}
    S = symmetric_gaussian_tensor(M, _rng(cfg, STREAM_S))
    ar = np.arange(M)
    S[ar, ar, ar, ar] += 2.0
    info = {"zero_fraction": 0.0}
    if mask_frac > 0.0:
        keep, zf = mode_group_mask(M, mask_frac, _rng(cfg, STREAM_MASK))
        S *= keep
        info["zero_fraction"] = zf
    S /= np.abs(S).max()
    return S.astype(np.float32), info


# ----------------------------------------------------------------------------
# launch fields
# ----------------------------------------------------------------------------

def _symbols(n: int, fmt: str, rng: np.random.Generator) -> np.ndarray:
    if fmt == "qpsk":
        re = rng.integers(0, 2, n) * 2 - 1
        im = rng.integers(0, 2, n) * 2 - 1
        return (re + 1j * im) / math.sqrt(2.0)
    if fmt == "16qam":
        lv = np.array([-3.0, -1.0, 1.0, 3.0])
        re = lv[rng.integers(0, 4, n)]
        im = lv[rng.integers(0, 4, n)]
        return (re + 1j * im) / math.sqrt(10.0)
    raise ValueError(fmt)


def _raised_cosine(f: np.ndarray, Ts: float, rolloff: float) -> np.ndarray:
    """Raised-cosine (Nyquist) spectrum, unit passband, f in 1/ps."""
    af = np.abs(f)
    f1 = (1.0 - rolloff) / (2.0 * Ts)
    f2 = (1.0 + rolloff) / (2.0 * Ts)
    H = np.zeros_like(af)
    H[af <= f1] = 1.0
    mid = (af > f1) & (af <= f2)
    H[mid] = 0.5 * (1.0 + np.cos(np.pi * Ts / rolloff * (af[mid] - f1)))
    return H


def shaped_field(rng: np.random.Generator, M: int, T: int, sps: int, n_ch: int,
                 spacing_thz: float, fmt: str, power_per_ch: float,
                 rolloff: float = 0.1) -> tuple[np.ndarray, float]:
    """WDM comb of raised-cosine shaped symbol trains on every mode.

    The symbol train is zero-stuffed to ``sps`` samples per symbol and
    filtered with a raised-cosine spectrum (periodic in the window); channel c
    of n_ch sits at (c - (n_ch-1)/2) * spacing.  Each channel is scaled to
    ``power_per_ch`` watts average power.  Returns (field [M,T] complex128, dt).
    """
    Ts = 1.0 / BAUD_THZ
    dt = Ts / sps
    if T % sps:
        raise ValueError("T must be a multiple of samples per symbol")
    ns = T // sps
    f = np.fft.fftfreq(T, dt)
    H = _raised_cosine(f, Ts, rolloff)
    t = np.arange(T) * dt
    out = np.zeros((M, T), dtype=np.complex128)
    for p in range(M):
        for c in range(n_ch):
            x = np.zeros(T, dtype=np.complex128)
            x[::sps] = _symbols(ns, fmt, rng)
            y = np.fft.ifft(np.fft.fft(x) * H)
            fc = (c - (n_ch - 1) / 2.0) * spacing_thz
            y *= np.exp(2j * np.pi * fc * t)
            y *= math.sqrt(power_per_ch / np.mean(np.abs(y) ** 2))
            out[p] += y
    return out, dt


def _dbm(p_dbm: float) -> float:
    return 1e-3 * 10.0 ** (p_dbm / 10.0)


def _random_beta(M: int, cfg: int) -> np.ndarray:
    rng = _rng(cfg, STREAM_BETA)
    beta = np.zeros((M, 3))
    beta[:, 0] = rng.uniform(-1000.0, 1000.0, M)   # rad/km
    beta[:, 1] = rng.uniform(-500.0, 500.0, M)     # ps/km  (+-0.5 ps/m)
    beta[:, 2] = rng.uniform(-25.0, -15.0, M)      # ps^2/km
    return beta


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

def soliton_problem(T: int = 4096, window: float = 100.0, T0: float = 2.0,
                    beta2: float = -20.0, gamma: float = 1.3, h: float = 0.005,
                    n_steps: int = 200, noise: float = 1e-6, cfg: int = 0) -> Problem:
    """Fundamental sech soliton of the scalar equation (one mode)."""
    dt = window / T
    t = (np.arange(T) - T // 2) * dt
    P0 = abs(beta2) / (gamma * T0 * T0)
    A = math.sqrt(P0) / np.cosh(t / T0) + 0j
    if noise > 0.0:
        rng = _rng(cfg, STREAM_NOISE)
        A = A + noise * math.sqrt(P0) * (rng.standard_normal(T) + 1j * rng.standard_normal(T)) / math.sqrt(2.0)
    beta = np.array([[0.0, 0.0, beta2]])
    return Problem("soliton", A[None, :].astype(np.complex128), beta, np.zeros(1),
                   np.ones((1, 1, 1, 1), dtype=np.float32), gamma, dt, h, n_steps, True,
                   {"P0": P0, "T0": T0, "window": window})


def make_problem(name: str, T: int | None = None, n_steps: int | None = None,
                 M: int | None = None, tensor: tuple | None = None) -> Problem:
    """Build one of the named workloads; T, n_steps and M may be reduced for tests.
    ``tensor`` = (S, info) of an earlier call with the same name and M skips
    regenerating the coupling tensor (it does not depend on T)."""
    if name == "soliton":
        kw = {}
        if T is not None:
            kw["T"] = T
        if n_steps is not None:
            kw["n_steps"] = n_steps
        return soliton_problem(**kw)
    if name == "manakov":
        return manakov_problem(M=M or 30, T=T or 2 ** 16, n_steps=n_steps or 100)
    if name == "qpsk6":
        cfg, M = 1, (M or 6)
        T = T or 2 ** 14
        A, dt = shaped_field(_rng(cfg, STREAM_SYMBOLS), M, T, 8, 1, 0.05, "qpsk", _dbm(0.0))
        S, info = tensor if tensor is not None else coupling_tensor(M, cfg)
        return Problem(name, A.astype(np.complex64), _random_beta(M, cfg), np.zeros(M), S, 1.0,
                       dt, 0.1, n_steps or 100, True, info)
    if name == "wdm36":
        cfg, M = 2, (M or 36)
        T = T or 2 ** 16
        A, dt = shaped_field(_rng(cfg, STREAM_SYMBOLS), M, T, 32, 8, 0.05, "16qam", _dbm(-2.0))
        S, info = tensor if tensor is not None else coupling_tensor(M, cfg, mask_frac=0.7)
        return Problem(name, A.astype(np.complex64), _random_beta(M, cfg), np.zeros(M), S, 1.0,
                       dt, 0.05, n_steps or 1000, True, info)
    if name == "wdm120":
        cfg, M = 4, (M or 120)
        T = T or 2 ** 17
        A, dt = shaped_field(_rng(cfg, STREAM_SYMBOLS), M, T, 16, 4, 0.05, "qpsk", _dbm(-3.0))
        S, info = tensor if tensor is not None else coupling_tensor(M, cfg)
        return Problem(name, A.astype(np.complex64), table3_beta(M), np.zeros(M), S, 0.5,
                       dt, 0.02, n_steps or 500, True, info)
    raise ValueError(f"unknown workload {name!r}")


def xpm_matrix(M: int, rng: np.random.Generator) -> np.ndarray:
    """Synthetic symmetric XPM coupling matrix: kappa_aa = 1 (intramodal),
    kappa_ab ~ U(0.2, 0.7) for a != b (intermodal), FP32."""
    k = rng.uniform(0.2, 0.7, (M, M))
    k = np.triu(k, 1)
    k = k + k.T + np.eye(M)
    return k.astype(np.float32)


def manakov_problem(M: int = 30, T: int = 2 ** 14, n_steps: int = 100, cfg: int = 5) -> Problem:
    """The paper's own model (Eq. 1, Manakov / XPM form): M rows (spatial modes x 2
    polarizations), 8-channel 16-QAM WDM per row at -2 dBm/channel, 32 samples per
    symbol, beta from Table 3 per mode group (two rows per spatial mode), the
    paper's attenuation 0.23 dB/km and gamma = 0.61 /W/km, h = 100 m."""
    A, dt = shaped_field(_rng(cfg, STREAM_SYMBOLS), M, T, 32, 8, 0.05, "16qam", _dbm(-2.0))
    spatial = (M + 1) // 2
    beta = np.repeat(table3_beta(spatial), 2, axis=0)[:M]
    alpha = np.full(M, 0.23 * math.log(10.0) / 10.0)   # dB/km -> 1/km (power)
    kappa = xpm_matrix(M, _rng(cfg, STREAM_S))
    return Problem("manakov", A.astype(np.complex64), beta, alpha, None, 0.61, dt, 0.1, n_steps,
                   False, {"model": "Eq. (1) Manakov/XPM"}, kappa)


# ----------------------------------------------------------------------------
# serving stream
# ----------------------------------------------------------------------------

@dataclass
class RequestSpec:
    index: int
    arrival: float      # seconds after stream start
    M: int
    T: int
    L: float            # km
    style: str          # "qpsk6" (M in {1,6}) or "wdm36" (M in {15,36})


def serving_stream(n: int = 256, rate: float | None = None, cfg: int = 3) -> list[RequestSpec]:
    """Poisson request stream; rate=None puts every arrival at t=0 (saturated)."""
    rng = _rng(cfg, STREAM_ARRIVALS)
    Ms = rng.choice([1, 6, 15, 36], n)
    Ts = rng.choice([2 ** 12, 2 ** 14, 2 ** 16], n)
    Ls = rng.choice([1.0, 10.0, 50.0], n)
    if rate is None:
        arr = np.zeros(n)
    else:
        arr = np.cumsum(_rng(cfg, STREAM_ARRIVALS, 1).exponential(1.0 / rate, n))
    return [RequestSpec(i, float(arr[i]), int(Ms[i]), int(Ts[i]), float(Ls[i]),
                        "qpsk6" if Ms[i] <= 6 else "wdm36") for i in range(n)]


_TENSOR_CACHE: dict = {}


def _request_tensor(M: int, cfg: int, masked: bool):
    """Requests of one mode count share one fiber's tensor (generated once)."""
    key = (M, cfg, masked)
    if key not in _TENSOR_CACHE:
        _TENSOR_CACHE[key] = coupling_tensor(M, cfg * 100 + M, mask_frac=0.7 if masked else 0.0)
    return _TENSOR_CACHE[key]


def request_problem(spec: RequestSpec, cfg: int = 3) -> Problem:
    """Field and coefficients of one serving request (seeded by its index)."""
    sub = 1000 + spec.index
    M, T = spec.M, spec.T
    if spec.style == "qpsk6":
        A, dt = shaped_field(_rng(cfg, STREAM_SYMBOLS, sub), M, T, 8, 1, 0.05, "qpsk", _dbm(0.0))
        S, info = _request_tensor(M, cfg, False)
        h = 0.1
        beta = _random_beta(M, cfg * 100000 + sub)
    else:
        A, dt = shaped_field(_rng(cfg, STREAM_SYMBOLS, sub), M, T, 32, 8, 0.05, "16qam", _dbm(-2.0))
        S, info = _request_tensor(M, cfg, True)
        h = 0.05
        beta = _random_beta(M, cfg * 100000 + sub)
    n_steps = int(round(spec.L / h))
    return Problem(f"req{spec.index}", A.astype(np.complex64), beta, np.zeros(M), S, 1.0, dt, h,
                   n_steps, True, info)
