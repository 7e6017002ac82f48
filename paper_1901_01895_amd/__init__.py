"""Python binding of libmmnlse (ctypes), RK4IP for coupled multimode NLSEs on MI355X.

Argument marshalling only: every step of the propagation runs in the HIP
library.  PyTorch supplies device memory and the stream.  The library must
have been built (``python -m paper_1901_01895_amd.build``); loading fails
loudly otherwise, there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmmnlse.so")

FP32, SPLIT_BF16, SPLIT_BF16_S = 0, 1, 2
RK4IP, SSFM_RK4, SSFM_AGRAWAL = 0, 1, 2
C64, C128 = 0, 1
S_SYMMETRIC, KERR_GENERIC, KERR_MANAKOV = 0x1, 0x2, 0x4
KERR_PATHS = {0: "small", 1: "tiled", 2: "mfma", 3: "manakov"}

STATUS = {0: "OK", 1: "E_INVALID", 2: "E_NOMEM", 3: "E_DEVICE", 4: "E_NONFINITE", 5: "E_BUSY",
          6: "E_UNSUPPORTED", 7: "E_STEP"}

SYMBOLS = (
    "mmnlse_create", "mmnlse_destroy", "mmnlse_last_error", "mmnlse_propagate", "mmnlse_advance",
    "mmnlse_amplify", "mmnlse_linear_half_step", "mmnlse_kerr", "mmnlse_power", "mmnlse_power_noalloc",
    "mmnlse_step_doubling",
    "mmnlse_synchronize", "mmnlse_footprint", "mmnlse_kerr_path", "mmnlse_profile",
    "mmnlse_propagate_adaptive", "mmnlse_kerr_work", "mmnlse_kerr_plan",
    "mmnlse_server_create", "mmnlse_server_submit", "mmnlse_server_poll", "mmnlse_server_wait",
    "mmnlse_server_stats", "mmnlse_server_destroy",
)


class MMNLSEError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_int32), ("T", ctypes.c_int32), ("dt_ps", ctypes.c_double),
        ("n_beta", ctypes.c_int32), ("beta", ctypes.POINTER(ctypes.c_double)),
        ("alpha", ctypes.POINTER(ctypes.c_double)), ("S", ctypes.POINTER(ctypes.c_float)),
        ("gamma", ctypes.c_double), ("h_km", ctypes.c_double), ("L_km", ctypes.c_double),
        ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32),
        ("kappa", ctypes.POINTER(ctypes.c_float)), ("method", ctypes.c_int32),
        ("diag_every", ctypes.c_int32), ("span_km", ctypes.c_double),
    ]


class ServerConfig(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_size_t), ("max_active", ctypes.c_int32),
                ("n_streams", ctypes.c_int32), ("steps_per_tick", ctypes.c_int32)]


class ServerCounters(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("queued", ctypes.c_int32), ("active", ctypes.c_int32),
                ("admitted_bytes", ctypes.c_size_t), ("peak_admitted_bytes", ctypes.c_size_t),
                ("rounds", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("power_in", ctypes.c_double), ("power_out", ctypes.c_double),
                ("seconds", ctypes.c_double), ("steps", ctypes.c_int64),
                ("power_drift_max", ctypes.c_double), ("local_err_max", ctypes.c_double),
                ("diag_points", ctypes.c_int64)]


class AdaptiveConfig(ctypes.Structure):
    _fields_ = [("length_km", ctypes.c_double), ("tol", ctypes.c_double), ("h_init_km", ctypes.c_double),
                ("h_min_km", ctypes.c_double), ("h_max_km", ctypes.c_double),
                ("max_trials", ctypes.c_int64)]


class Trial(ctypes.Structure):
    _fields_ = [("z_km", ctypes.c_double), ("h_km", ctypes.c_double), ("delta", ctypes.c_double),
                ("accepted", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class AdaptiveResult(ctypes.Structure):
    _fields_ = [("z_km", ctypes.c_double), ("h_next_km", ctypes.c_double), ("accepted", ctypes.c_int64),
                ("rejected", ctypes.c_int64), ("trials", ctypes.c_int64), ("seconds", ctypes.c_double)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_1901_01895_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    lib.mmnlse_create.argtypes = [ctypes.POINTER(Config), vp, ctypes.POINTER(vp)]
    lib.mmnlse_destroy.argtypes = [vp]
    lib.mmnlse_last_error.restype = ctypes.c_char_p
    lib.mmnlse_last_error.argtypes = []
    lib.mmnlse_propagate.argtypes = [vp, vp, vp, i32, i32, ctypes.POINTER(Stats)]
    lib.mmnlse_advance.argtypes = [vp, vp, i64]
    lib.mmnlse_amplify.argtypes = [vp, vp]
    lib.mmnlse_linear_half_step.argtypes = [vp, vp, vp]
    lib.mmnlse_kerr.argtypes = [vp, vp, vp]
    lib.mmnlse_power.argtypes = [vp, vp, dp]
    lib.mmnlse_power_noalloc.argtypes = [vp, i64, ctypes.c_double, vp, vp]
    lib.mmnlse_step_doubling.argtypes = [vp, vp, dp]
    lib.mmnlse_synchronize.argtypes = [vp]
    lib.mmnlse_footprint.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.mmnlse_kerr_path.argtypes = [vp, ctypes.POINTER(i32)]
    lib.mmnlse_kerr_work.argtypes = [vp, dp]
    ip = ctypes.POINTER(ctypes.c_int32)
    lib.mmnlse_kerr_plan.argtypes = [ctypes.POINTER(ctypes.c_float), i32, i32, ip, ip, ip, ip, ip, dp]
    lib.mmnlse_profile.argtypes = [vp, vp, i64, dp, ctypes.POINTER(ctypes.c_int64)]
    lib.mmnlse_propagate_adaptive.argtypes = [vp, vp, ctypes.POINTER(AdaptiveConfig), ctypes.POINTER(Trial),
                                              i64, ctypes.POINTER(AdaptiveResult)]
    lib.mmnlse_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    lib.mmnlse_server_submit.argtypes = [vp, ctypes.POINTER(Config), vp, i32, ctypes.POINTER(ctypes.c_uint64)]
    for fn in (lib.mmnlse_server_poll, lib.mmnlse_server_wait):
        fn.argtypes = [vp, ctypes.c_uint64, vp, ctypes.POINTER(Stats), dp]
    lib.mmnlse_server_stats.argtypes = [vp, ctypes.POINTER(ServerCounters)]
    lib.mmnlse_server_destroy.argtypes = [vp]
    for name in SYMBOLS:
        if name != "mmnlse_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        raise MMNLSEError(status, load().mmnlse_last_error().decode())


def _dptr(x) -> int:
    """Device pointer of a contiguous complex64 CUDA tensor."""
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.complex64 and x.is_contiguous()):
        raise TypeError("expected a contiguous complex64 device tensor")
    return x.data_ptr()


def power_noalloc(X, dt: float, out, stream=None) -> None:
    """mmnlse_power_noalloc: writes dt * sum |X|^2 (FP64) into the one-element
    float64 device tensor ``out``, asynchronously on ``stream`` (default:
    torch's current stream), without allocating device memory."""
    import torch
    if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64 and out.numel() >= 1):
        raise TypeError("out must be a float64 device tensor")
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(load().mmnlse_power_noalloc(ctypes.c_void_p(_dptr(X)), int(X.numel()), float(dt),
                                       ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(s.cuda_stream)))


def make_config(M, T, dt, beta, S, gamma, h, L, alpha=None, precision=FP32, symmetric=None,
                generic=False, kappa=None, method=RK4IP, diag_every=0, span=0.0):
    """mmnlse_config for the arguments; returns (config, arrays it points into).

    With ``kappa`` ([M, M]) the paper's Manakov / XPM nonlinear operator of
    Eq. (1) is used and S is ignored (may be None).  ``span`` > 0 (km) puts a
    loss-compensating amplifier after every span."""
    beta = np.ascontiguousarray(np.asarray(beta, dtype=np.float64).reshape(M, -1))
    alpha = None if alpha is None else np.ascontiguousarray(np.asarray(alpha, dtype=np.float64))
    if kappa is not None:
        kappa = np.ascontiguousarray(np.asarray(kappa, dtype=np.float32).reshape(M, M))
        S, symmetric = None, False
    else:
        S = np.ascontiguousarray(np.asarray(S, dtype=np.float32).reshape(M, M, M, M))
        if symmetric is None:
            symmetric = bool(np.array_equal(S, S.transpose(0, 2, 1, 3)) and np.array_equal(S, S.transpose(3, 1, 2, 0)))
    cfg = Config()
    cfg.M, cfg.T, cfg.dt_ps = M, T, float(dt)
    cfg.n_beta = beta.shape[1]
    cfg.beta = beta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    cfg.alpha = alpha.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if alpha is not None else None
    cfg.S = S.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if S is not None else None
    cfg.kappa = kappa.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if kappa is not None else None
    cfg.gamma, cfg.h_km, cfg.L_km = float(gamma), float(h), float(L)
    cfg.precision = int(precision)
    cfg.method = int(method)
    cfg.diag_every = int(diag_every)
    cfg.span_km = float(span)
    cfg.flags = ((S_SYMMETRIC if symmetric else 0) | (KERR_GENERIC if generic else 0)
                 | (KERR_MANAKOV if kappa is not None else 0))
    return cfg, (beta, S, alpha, kappa)


def problem_config(p, precision=FP32, generic=False, L=None, method=RK4IP, diag_every=0, span=0.0):
    """mmnlse_config for a workloads.Problem."""
    return make_config(p.M, p.T, p.dt, p.beta, p.S, p.gamma, p.h, p.L if L is None else L,
                       p.alpha if np.any(p.alpha) else None, precision, p.symmetric, generic,
                       getattr(p, "kappa", None), method, diag_every, span)


def kerr_plan(S, precision: int = FP32) -> dict:
    """Host-only plan of the matrix-core contraction for tensor S [M,M,M,M]
    (mmnlse_kerr_plan): column positions and row slots (natural pair index,
    -1 for padding), passes of row tiles and their k-lists."""
    lib = load()
    S = np.ascontiguousarray(np.asarray(S, dtype=np.float32))
    M = S.shape[0]
    sp = S.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    counts = np.zeros(7, np.int32)
    cp = counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    _check(lib.mmnlse_kerr_plan(sp, M, int(precision), cp, None, None, None, None, None))
    P, Ppad, npass, nk_list, kw, rtm, nrt = (int(x) for x in counts)
    perm = np.zeros(Ppad, np.int32)
    rows = np.zeros(32 * nrt, np.int32)
    passes = np.zeros((max(npass, 1), 4), np.int32)
    klist = np.zeros(max(nk_list, 1), np.int32)
    entries = np.zeros(3, np.float64)
    ptr = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    _check(lib.mmnlse_kerr_plan(sp, M, int(precision), cp, ptr(perm), ptr(rows), ptr(passes), ptr(klist),
                                entries.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return {"P": P, "Ppad": Ppad, "kw": kw, "rtm": rtm, "nrt": nrt, "perm": perm, "rows": rows,
            "passes": passes[:npass], "klist": klist[:nk_list],
            "entries": {"dense": entries[0], "multiplied": entries[1], "nonzero": entries[2]}}


class Propagator:
    """One RK4IP plan: fixed M, T, coefficients, tensor, h and L.

    Parameters mirror ``mmnlse_config``; ``stream`` is a torch.cuda.Stream
    (default: torch's current stream).
    """

    def __init__(self, M: int, T: int, dt: float, beta, S, gamma: float, h: float, L: float,
                 alpha=None, precision: int = FP32, symmetric: bool | None = None,
                 generic: bool = False, stream=None, kappa=None, method: int = RK4IP,
                 diag_every: int = 0, span: float = 0.0):
        import torch
        lib = load()
        cfg, self._keep = make_config(M, T, dt, beta, S, gamma, h, L, alpha, precision, symmetric, generic,
                                      kappa, method, diag_every, span)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        handle = ctypes.c_void_p()
        _check(lib.mmnlse_create(ctypes.byref(cfg), ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(handle)))
        self._h = handle
        self.M, self.T, self.dt, self.h, self.L = M, T, dt, h, L
        self.n_steps = int(round(L / h))
        self.precision = precision

    @classmethod
    def from_problem(cls, p, precision: int = FP32, generic: bool = False, L: float | None = None,
                     stream=None, method: int = RK4IP, diag_every: int = 0, span: float = 0.0):
        return cls(p.M, p.T, p.dt, p.beta, p.S, p.gamma, p.h, p.L if L is None else L,
                   alpha=p.alpha if np.any(p.alpha) else None, precision=precision,
                   symmetric=p.symmetric, generic=generic, stream=stream,
                   kappa=getattr(p, "kappa", None), method=method, diag_every=diag_every, span=span)

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            load().mmnlse_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------
    def propagate(self, A, stats: bool = False):
        """Propagate over L.  numpy input -> numpy output (host path);
        torch device tensor (complex64/complex128) -> new device tensor."""
        lib = load()
        st = Stats()
        if isinstance(A, np.ndarray):
            dtype = C128 if A.dtype == np.complex128 else C64
            src = np.ascontiguousarray(A, dtype=np.complex128 if dtype == C128 else np.complex64)
            out = np.empty_like(src)
            _check(lib.mmnlse_propagate(self._h, src.ctypes.data_as(ctypes.c_void_p),
                                        out.ctypes.data_as(ctypes.c_void_p), dtype, 0, ctypes.byref(st)))
        else:
            import torch
            dtype = C128 if A.dtype == torch.complex128 else C64
            if A.dtype not in (torch.complex64, torch.complex128) or not A.is_cuda:
                raise TypeError("expected a complex64/complex128 device tensor")
            src = A.contiguous()
            out = torch.empty_like(src)
            _check(lib.mmnlse_propagate(self._h, ctypes.c_void_p(src.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), dtype, 1, ctypes.byref(st)))
        if stats:
            return out, {"power_in": st.power_in, "power_out": st.power_out, "seconds": st.seconds,
                         "steps": st.steps, "power_drift_max": st.power_drift_max,
                         "local_err_max": st.local_err_max, "diag_points": st.diag_points}
        return out

    def advance(self, A, n_steps: int):
        """In-place device advance by n_steps (asynchronous on the plan's stream)."""
        _check(load().mmnlse_advance(self._h, ctypes.c_void_p(_dptr(A)), int(n_steps)))
        return A

    def amplify(self, A):
        """In-place span-end amplifier exp(alpha_p span / 2) per mode (asynchronous)."""
        _check(load().mmnlse_amplify(self._h, ctypes.c_void_p(_dptr(A))))
        return A

    def linear_half_step(self, X, Y=None):
        import torch
        Y = torch.empty_like(X) if Y is None else Y
        _check(load().mmnlse_linear_half_step(self._h, ctypes.c_void_p(_dptr(X)), ctypes.c_void_p(_dptr(Y))))
        return Y

    def kerr(self, X, Y=None):
        import torch
        Y = torch.empty_like(X) if Y is None else Y
        _check(load().mmnlse_kerr(self._h, ctypes.c_void_p(_dptr(X)), ctypes.c_void_p(_dptr(Y))))
        return Y

    def power(self, X) -> float:
        out = ctypes.c_double()
        _check(load().mmnlse_power(self._h, ctypes.c_void_p(_dptr(X)), ctypes.byref(out)))
        return out.value

    def step_doubling(self, X) -> float:
        out = ctypes.c_double()
        _check(load().mmnlse_step_doubling(self._h, ctypes.c_void_p(_dptr(X)), ctypes.byref(out)))
        return out.value

    def propagate_adaptive(self, A, length: float, tol: float, h_init: float, h_min: float = 0.0,
                           h_max: float = 0.0, max_trials: int = 100000, log_cap: int = 100000):
        """Adaptive-step propagation of device field A in place (mmnlse_propagate_adaptive).

        Returns (result dict, trials) with trials a list of (z, h, delta, accepted)
        tuples.  On E_STEP raises MMNLSEError whose ``result`` and ``trials``
        attributes hold the same for the part that was covered.
        """
        ac = AdaptiveConfig(float(length), float(tol), float(h_init), float(h_min), float(h_max),
                            int(max_trials))
        log = (Trial * max(int(log_cap), 1))()
        res = AdaptiveResult()
        st = load().mmnlse_propagate_adaptive(self._h, ctypes.c_void_p(_dptr(A)), ctypes.byref(ac), log,
                                              int(log_cap), ctypes.byref(res))
        out = {k: getattr(res, k) for k, _ in AdaptiveResult._fields_}
        trials = [(t.z_km, t.h_km, t.delta, bool(t.accepted)) for t in log[:min(res.trials, int(log_cap))]]
        if st != 0:
            err = MMNLSEError(st, load().mmnlse_last_error().decode())
            err.result, err.trials = out, trials
            raise err
        return out, trials

    def kerr_work(self) -> dict:
        """Packed-tensor entries per sample of one Kerr evaluation (matrix-core path):
        dense P*P, multiplied (nonzero blocks), nonzero."""
        out = (ctypes.c_double * 3)()
        _check(load().mmnlse_kerr_work(self._h, out))
        return {"dense": out[0], "multiplied": out[1], "nonzero": out[2]}

    def profile(self, A, n_steps: int) -> dict:
        """Advance A in place by n_steps with HIP events around every launch;
        returns summed device milliseconds and launch counts per kernel class."""
        ms = (ctypes.c_double * 2)()
        cnt = (ctypes.c_int64 * 3)()
        _check(load().mmnlse_profile(self._h, ctypes.c_void_p(_dptr(A)), int(n_steps), ms, cnt))
        return {"kerr_ms": ms[0], "linear_ms": ms[1], "kerr_launches": cnt[0],
                "linear_launches": cnt[1], "kerr_evals": cnt[2]}

    def synchronize(self):
        _check(load().mmnlse_synchronize(self._h))

    @property
    def footprint(self) -> int:
        out = ctypes.c_size_t()
        _check(load().mmnlse_footprint(self._h, ctypes.byref(out)))
        return out.value

    @property
    def kerr_path(self) -> str:
        out = ctypes.c_int32()
        _check(load().mmnlse_kerr_path(self._h, ctypes.byref(out)))
        return KERR_PATHS[out.value]


class Server:
    """Continuous-batching server (mmnlse_server_*): submit host fields, poll results."""

    def __init__(self, mem_budget_bytes: int = 0, max_active: int = 0, n_streams: int = 0,
                 steps_per_tick: int = 0):
        lib = load()
        c = ServerConfig(mem_budget_bytes, max_active, n_streams, steps_per_tick)
        h = ctypes.c_void_p()
        _check(lib.mmnlse_server_create(ctypes.byref(c), ctypes.byref(h)))
        self._h = h
        self._pending = {}

    def submit(self, A: np.ndarray, cfg_and_keep) -> int:
        """Queue a propagation; cfg_and_keep from make_config/problem_config."""
        cfg, keep = cfg_and_keep
        dtype = C128 if A.dtype == np.complex128 else C64
        A = np.ascontiguousarray(A, dtype=np.complex128 if dtype == C128 else np.complex64)
        t = ctypes.c_uint64()
        _check(load().mmnlse_server_submit(self._h, ctypes.byref(cfg), A.ctypes.data_as(ctypes.c_void_p),
                                           dtype, ctypes.byref(t)))
        self._pending[t.value] = (np.empty_like(A), keep)
        return t.value

    def _finish(self, ticket, block):
        out = self._pending.get(ticket, (None, None))[0]
        st, lat = Stats(), ctypes.c_double()
        fn = load().mmnlse_server_wait if block else load().mmnlse_server_poll
        ptr = out.ctypes.data_as(ctypes.c_void_p) if out is not None else None
        r = fn(self._h, ticket, ptr, ctypes.byref(st), ctypes.byref(lat))
        if r == 5:  # E_BUSY
            return None
        self._pending.pop(ticket, None)
        _check(r)
        return out, {"power_in": st.power_in, "power_out": st.power_out, "seconds": st.seconds,
                     "steps": st.steps, "latency": lat.value}

    def poll(self, ticket: int):
        """(field, info) once done, else None."""
        return self._finish(ticket, False)

    def wait(self, ticket: int):
        return self._finish(ticket, True)

    def counters(self) -> dict:
        c = ServerCounters()
        _check(load().mmnlse_server_stats(self._h, ctypes.byref(c)))
        return {k: getattr(c, k) for k, _ in ServerCounters._fields_}

    def close(self):
        if getattr(self, "_h", None):
            load().mmnlse_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
