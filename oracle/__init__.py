"""ctypes front end of the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are its only users.  The product path never imports it.

Each wrapper converts numpy arrays to contiguous buffers and calls the C
function of the same name; see ``oracle.h`` for the definitions (Sec. 2.1 of
the paper, step by step).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_float_p = ctypes.POINTER(ctypes.c_float)
_c_u8_p = ctypes.POINTER(ctypes.c_uint8)
_c_i8_p = ctypes.POINTER(ctypes.c_int8)
_c_i32_p = ctypes.POINTER(ctypes.c_int32)
_c_i64_p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C99, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        L.oracle_sample10.argtypes = [_c_u8_p, ctypes.c_int64]
        L.oracle_sample10.restype = ctypes.c_int32
        L.oracle_unpack10.argtypes = [_c_u8_p, ctypes.c_int64, ctypes.c_int64, _c_i32_p]
        L.oracle_unpack10.restype = None
        L.oracle_split_delay.argtypes = [ctypes.c_double, ctypes.c_int64, _c_i64_p, _c_double_p]
        L.oracle_split_delay.restype = ctypes.c_int
        L.oracle_pfb_fir.argtypes = [_c_double_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                     ctypes.c_int, _c_float_p, ctypes.c_int64, ctypes.c_int64,
                                     _c_double_p]
        L.oracle_pfb_fir.restype = ctypes.c_int
        L.oracle_fft.argtypes = [_c_double_p, _c_double_p, ctypes.c_int]
        L.oracle_fft.restype = ctypes.c_int
        L.oracle_rfft_keep.argtypes = [_c_double_p, ctypes.c_int, _c_double_p]
        L.oracle_rfft_keep.restype = ctypes.c_int
        L.oracle_fine_delay_gain.argtypes = [_c_double_p, ctypes.c_int, ctypes.c_double,
                                             ctypes.c_double, _c_float_p, _c_double_p]
        L.oracle_fine_delay_gain.restype = None
        L.oracle_quantize.argtypes = [ctypes.c_double]
        L.oracle_quantize.restype = ctypes.c_int8
        L.oracle_heap_layout.argtypes = [_c_i8_p, ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                         ctypes.c_int, _c_i8_p]
        L.oracle_heap_layout.restype = ctypes.c_int
        L.oracle_channelize.argtypes = [_c_u8_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int64, _c_float_p, _c_double_p,
                                        _c_double_p, _c_float_p, ctypes.c_int64, ctypes.c_int64,
                                        _c_double_p, _c_double_p, _c_double_p, _c_i8_p, _c_i8_p]
        L.oracle_channelize.restype = ctypes.c_int64
        _lib = L
    return _lib


def _p(a, ctype):
    return a.ctypes.data_as(ctype)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def unpack10(raw, first: int = 0, count: int | None = None) -> np.ndarray:
    if isinstance(raw, (bytes, bytearray)):
        raw = np.frombuffer(raw, dtype=np.uint8)
    raw = _c(raw, np.uint8)
    if count is None:
        count = raw.size * 8 // 10 - first
    out = np.empty(count, dtype=np.int32)
    lib().oracle_unpack10(_p(raw, _c_u8_p), first, count, _p(out, _c_i32_p))
    return out


def split_delay(d: float, max_delay: int):
    """(valid, coarse, fine) of the total delay ``d``."""
    c = ctypes.c_int64()
    t = ctypes.c_double()
    ok = lib().oracle_split_delay(float(d), int(max_delay), ctypes.byref(c), ctypes.byref(t))
    return bool(ok), int(c.value), float(t.value)


def fft(x) -> np.ndarray:
    x = np.asarray(x, dtype=np.complex128)
    re, im = _c(x.real, np.float64), _c(x.imag, np.float64)
    if lib().oracle_fft(_p(re, _c_double_p), _p(im, _c_double_p), x.size):
        raise ValueError("length must be a power of two")
    return re + 1j * im


def pfb_fir(s, n: int, taps: int, h, F: int, coarse: int, s_first: int = 0) -> np.ndarray:
    s, h = _c(s, np.float64), _c(h, np.float32)
    g = np.empty(2 * n, dtype=np.float64)
    if lib().oracle_pfb_fir(_p(s, _c_double_p), s_first, s.size, n, taps, _p(h, _c_float_p),
                            F, coarse, _p(g, _c_double_p)):
        raise ValueError("window outside the supplied samples")
    return g


def rfft_keep(g) -> np.ndarray:
    g = _c(g, np.float64)
    n = g.size // 2
    X = np.empty(2 * n, dtype=np.float64)
    if lib().oracle_rfft_keep(_p(g, _c_double_p), n, _p(X, _c_double_p)):
        raise ValueError("length must be a power of two")
    return X[0::2] + 1j * X[1::2]


def fine_delay_gain(X, tau: float, phi: float, gain) -> np.ndarray:
    X = np.asarray(X, dtype=np.complex128)
    n = X.size
    Xi = _c(np.stack([X.real, X.imag], -1), np.float64)
    gi = np.asarray(gain)
    if np.iscomplexobj(gi):
        gi = np.stack([gi.real, gi.imag], -1)
    gi = _c(gi, np.float32)
    Y = np.empty(2 * n, dtype=np.float64)
    lib().oracle_fine_delay_gain(_p(Xi, _c_double_p), n, float(tau), float(phi),
                                 _p(gi, _c_float_p), _p(Y, _c_double_p))
    return Y[0::2] + 1j * Y[1::2]


def quantize(v) -> np.ndarray:
    v = np.asarray(v, dtype=np.float64)
    f = lib().oracle_quantize
    return np.array([f(float(x)) for x in v.ravel()], dtype=np.int8).reshape(v.shape)


def heap_layout(q, S: int) -> np.ndarray:
    """q int8 [A][2][M][n][2] -> heap int8 [A][M/S][n][S][2][2]."""
    q = _c(q, np.int8)
    A, _, M, n, _ = q.shape
    out = np.empty((A, M // S, n, S, 2, 2), dtype=np.int8)
    if lib().oracle_heap_layout(_p(q, _c_i8_p), A, M, n, S, _p(out, _c_i8_p)):
        raise ValueError("M must be a multiple of S")
    return out


def channelize(raw, total: int, n: int, taps: int, max_delay: int, weights, delays, phases,
               gains, f_begin: int = 0, f_end: int | None = None,
               want=("y", "q", "valid")) -> dict:
    """Run the whole path for spectra [f_begin, f_end); see ``oracle.h``.

    Returns a dict with the requested members of g, x, y (complex128), q
    (int8 [A][2][nF][n][2]) and valid, plus ``invalid`` (count).
    """
    raw = _c(raw, np.uint8)
    A = raw.shape[0]
    M = total // (2 * n)
    f_end = M if f_end is None else f_end
    nF = f_end - f_begin
    weights, gains = _c(weights, np.float32), _c(gains, np.float32)
    delays, phases = _c(delays, np.float64), _c(phases, np.float64)
    assert delays.shape == (A, 2, M) and phases.shape == (A, 2, M)
    assert gains.shape == (A, 2, n, 2) and weights.size == 2 * n * taps
    bufs = {}
    if "g" in want:
        bufs["g"] = np.empty((A, 2, nF, 2 * n), dtype=np.float64)
    for k in ("x", "y"):
        if k in want:
            bufs[k] = np.empty((A, 2, nF, n, 2), dtype=np.float64)
    if "q" in want:
        bufs["q"] = np.empty((A, 2, nF, n, 2), dtype=np.int8)
    if "valid" in want:
        bufs["valid"] = np.empty((A, 2, nF), dtype=np.int8)
    nul_d, nul_i8 = _c_double_p(), _c_i8_p()
    rc = lib().oracle_channelize(
        _p(raw, _c_u8_p), total, A, n, taps, max_delay, _p(weights, _c_float_p),
        _p(delays, _c_double_p), _p(phases, _c_double_p), _p(gains, _c_float_p),
        f_begin, f_end,
        _p(bufs["g"], _c_double_p) if "g" in bufs else nul_d,
        _p(bufs["x"], _c_double_p) if "x" in bufs else nul_d,
        _p(bufs["y"], _c_double_p) if "y" in bufs else nul_d,
        _p(bufs["q"], _c_i8_p) if "q" in bufs else nul_i8,
        _p(bufs["valid"], _c_i8_p) if "valid" in bufs else nul_i8)
    if rc < 0:
        raise ValueError("oracle_channelize rejected its arguments")
    out = {"invalid": int(rc)}
    if "g" in bufs:
        out["g"] = bufs["g"]
    for k in ("x", "y"):
        if k in bufs:
            out[k] = bufs[k][..., 0] + 1j * bufs[k][..., 1]
    for k in ("q", "valid"):
        if k in bufs:
            out[k] = bufs[k]
    return out
