"""The C-ABI library: it loads and exports every symbol the header declares (CPU only)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mmnlse.h")
LIB = os.path.join(ROOT, "paper_1901_01895_amd", "libmmnlse.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mmnlse_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("mmnlse_create", "mmnlse_propagate", "mmnlse_destroy", "mmnlse_last_error",
              "mmnlse_advance", "mmnlse_linear_half_step", "mmnlse_kerr", "mmnlse_power",
              "mmnlse_step_doubling"):
        assert s in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_lists_every_declared_symbol():
    import paper_1901_01895_amd as mm
    assert sorted(mm.SYMBOLS) == declared_symbols()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_create_rejects_bad_arguments_without_touching_the_gpu():
    """Argument validation runs before any device call."""
    import numpy as np
    import paper_1901_01895_amd as mm
    lib = mm.load()
    S = np.ones((1, 1, 1, 1), np.float32)
    beta = np.zeros((1, 3))
    base = dict(M=1, T=4096, dt_ps=0.1, n_beta=3, gamma=1.0, h_km=0.1, L_km=1.0)

    def make(**kw):
        c = mm.Config()
        d = dict(base, **kw)
        for k, v in d.items():
            setattr(c, k, v)
        c.beta = beta.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        c.S = S.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        return c

    h = ctypes.c_void_p()
    for bad in (dict(T=1000), dict(T=32), dict(M=0), dict(L_km=1.05), dict(h_km=0.0),
                dict(dt_ps=-1.0), dict(precision=7), dict(n_beta=9), dict(method=5),
                dict(diag_every=-1), dict(T=2 ** 21), dict(M=257), dict(method=2),
                dict(span_km=-0.5), dict(span_km=float("nan")), dict(span_km=0.25), dict(span_km=0.3),
                dict(span_km=0.05)):
        c = make(**bad)
        assert lib.mmnlse_create(ctypes.byref(c), None, ctypes.byref(h)) == 1, bad
        assert lib.mmnlse_last_error()
    # split precision without a symmetric tensor is refused
    c = make(precision=1, flags=0)
    assert lib.mmnlse_create(ctypes.byref(c), None, ctypes.byref(h)) == 1
    assert lib.mmnlse_destroy(None) == 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_power_noalloc_rejects_bad_arguments_without_touching_the_gpu():
    """mmnlse_power_noalloc checks its arguments before any device call (the
    pointers below are never dereferenced)."""
    import paper_1901_01895_amd as mm
    lib = mm.load()
    x, o = ctypes.c_void_p(4096), ctypes.c_void_p(8192)
    for args in ((None, 64, 1.0, o), (x, 64, 1.0, None), (x, 0, 1.0, o), (x, -1, 1.0, o),
                 (x, (1 << 40) + 1, 1.0, o), (x, 64, 0.0, o), (x, 64, -2.0, o), (x, 64, float("nan"), o),
                 (x, 64, float("inf"), o), (ctypes.c_void_p(4100), 64, 1.0, o), (x, 64, 1.0, ctypes.c_void_p(8196))):
        assert lib.mmnlse_power_noalloc(*args, None) == 1, args
        assert lib.mmnlse_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_create_reports_host_memory_exhaustion_without_touching_the_gpu(monkeypatch):
    """A set-up whose host tables exceed MMNLSE_HOST_BYTES_LIMIT fails with
    E_NOMEM before any device call (the same status a std::bad_alloc in the
    set-up returns; nothing escapes the C boundary)."""
    import numpy as np
    import paper_1901_01895_amd as mm
    import workloads as W
    lib = mm.load()
    p = W.make_problem("wdm36", T=2 ** 10, n_steps=1)
    cfg, keep = mm.problem_config(p, precision=mm.SPLIT_BF16)
    monkeypatch.setenv("MMNLSE_HOST_BYTES_LIMIT", "100000")
    h = ctypes.c_void_p()
    assert lib.mmnlse_create(ctypes.byref(cfg), None, ctypes.byref(h)) == 2
    assert b"host memory" in lib.mmnlse_last_error()
    assert not h.value
