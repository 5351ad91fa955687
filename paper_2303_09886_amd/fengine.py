"""ctypes binding of ``libfengine.so`` (the C ABI in ``include/fengine.h``).

Argument marshalling only: every step of the channelizer runs in the HIP
kernels of the library.  Buffers are torch tensors on the GPU; their
``data_ptr()`` is handed to the library, which enqueues work on the HIP
stream the :class:`Stream` was bound to.  If the library is missing this
module raises: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

from . import build as _build

FE_OK, FE_EINVAL, FE_ENOMEM, FE_EHIP, FE_EDELAY, FE_ESIZE = 0, -1, -2, -3, -4, -5
FE_NOALLOC_SCRATCH_BYTES = 64 << 20         # include/fengine.h
FE_PREC_FP32, FE_PREC_FP16, FE_PREC_BF16 = 0, 1, 2
PRECISIONS = {"fp32": FE_PREC_FP32, "fp16": FE_PREC_FP16, "bf16": FE_PREC_BF16}
FE_PATH_AUTO, FE_PATH_SPLIT, FE_PATH_FUSED, FE_PATH_MATRIX_FIR, FE_PATH_SPLIT_FOLDED = 0, 1, 2, 3, 4
PATHS = {"auto": FE_PATH_AUTO, "split": FE_PATH_SPLIT, "fused": FE_PATH_FUSED, "matrix_fir": FE_PATH_MATRIX_FIR,
         "split_folded": FE_PATH_SPLIT_FOLDED}


class FEngineError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__("%s: %s (%d)" % (what, _strerror(status), status))


class _Config(ctypes.Structure):
    _fields_ = [("n_channels", ctypes.c_int32), ("taps", ctypes.c_int32),
                ("n_antennas", ctypes.c_int32), ("spectra_per_heap", ctypes.c_int32),
                ("max_delay", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("max_samples", ctypes.c_int64), ("weights", ctypes.POINTER(ctypes.c_float))]


class _Call(ctypes.Structure):
    _fields_ = [("raw", ctypes.c_void_p), ("n_samples", ctypes.c_int64), ("delays", ctypes.c_void_p),
                ("phases", ctypes.c_void_p), ("gains", ctypes.c_void_p), ("out", ctypes.c_void_p)]


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_st = ctypes.c_int32


def load_library(path: Optional[str] = None):
    """Load the built library (never builds; raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or _build.LIB
    if not os.path.exists(path):
        raise FEngineError(FE_EINVAL, "HIP library %s is not built (run "
                           "python -m paper_2303_09886_amd.build)" % path)
    L = ctypes.CDLL(path)
    L.fe_stream_create.argtypes = [ctypes.POINTER(_Config), _vp, ctypes.POINTER(_vp)]
    L.fe_stream_create.restype = _st
    L.fe_stream_destroy.argtypes = [_vp]
    L.fe_stream_destroy.restype = _st
    L.fe_stream_set_hip_stream.argtypes = [_vp, _vp]
    L.fe_stream_set_hip_stream.restype = _st
    L.fe_stream_reset.argtypes = [_vp]
    L.fe_stream_reset.restype = _st
    for name in ("fe_channelize", "fe_channelize_prequant", "fe_channelize_noalloc"):
        f = getattr(L, name)
        f.argtypes = [_vp, _vp, _i64, _vp, _vp, _vp, _vp]
        f.restype = _st
    L.fe_channelize_fir.argtypes = [_vp, _vp, _i64, _vp, _vp]
    L.fe_channelize_fir.restype = _st
    L.fe_stream_status.argtypes = [_vp]
    L.fe_stream_status.restype = _st
    L.fe_stream_timing.argtypes = [_vp, ctypes.c_int]
    L.fe_stream_timing.restype = _st
    L.fe_stream_timing_read.argtypes = [_vp, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)]
    L.fe_stream_timing_read.restype = _st
    L.fe_stream_autotune.argtypes = [_vp, _vp, _i64, _vp, _vp, _vp, _vp, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int)]
    L.fe_stream_autotune.restype = _st
    L.fe_stream_set_tuning.argtypes = [_vp, ctypes.c_int]
    L.fe_stream_set_tuning.restype = _st
    L.fe_stream_set_fft_parts.argtypes = [_vp, ctypes.c_int]
    L.fe_stream_set_fft_parts.restype = _st
    L.fe_stream_get_fft_parts.argtypes = [_vp, ctypes.POINTER(ctypes.c_int)]
    L.fe_stream_get_fft_parts.restype = _st
    L.fe_stream_set_schedule.argtypes = [_vp, ctypes.c_int, ctypes.c_int]
    L.fe_stream_set_schedule.restype = _st
    L.fe_stream_get_schedule.argtypes = [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.fe_stream_get_schedule.restype = _st
    L.fe_batch_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, _vp, ctypes.POINTER(_vp)]
    L.fe_batch_create.restype = _st
    L.fe_batch_destroy.argtypes = [_vp]
    L.fe_batch_destroy.restype = _st
    for name in ("fe_batch_run", "fe_batch_capture"):
        f = getattr(L, name)
        f.argtypes = [_vp, ctypes.POINTER(_Call)]
        f.restype = _st
    L.fe_batch_launch.argtypes = [_vp]
    L.fe_batch_launch.restype = _st
    L.fe_batch_set_grouped.argtypes = [_vp, ctypes.c_int]
    L.fe_batch_set_grouped.restype = _st
    L.fe_debug_unpack10.argtypes = [_vp, _i64, _i64, _vp, _vp]
    L.fe_debug_unpack10.restype = _st
    L.fe_strerror.argtypes = [_st]
    L.fe_strerror.restype = ctypes.c_char_p
    L.fe_version.argtypes = []
    L.fe_version.restype = ctypes.c_int32
    _lib = L
    return L


def _strerror(status: int) -> str:
    try:
        return load_library().fe_strerror(status).decode()
    except Exception:
        return "status"


def _check(status: int, what: str):
    if status != FE_OK:
        raise FEngineError(status, what)


def version() -> int:
    return int(load_library().fe_version())


def _ptr(t, dtype, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a torch tensor on the GPU" % what)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (what, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    return ctypes.c_void_p(t.data_ptr())


def _hip_stream(stream) -> ctypes.c_void_p:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _need(t, count, what):
    """Refuse a buffer smaller than the header's layout needs: the kernels
    would read or write past its end."""
    if t.numel() < count:
        raise ValueError("%s holds %d elements, the call needs %d" % (what, t.numel(), count))


def call_sizes(n_antennas: int, n_channels: int, n_samples: int) -> dict:
    """Element counts one call needs (include/fengine.h): raw uint8
    [A][2][N*5/4], delays and phases float64 [A][2][M], gains float32
    [A][2][n][2], and each output (int8 heaps, float32 spectra or filtered
    samples) 2*A*N elements."""
    N = int(n_samples)
    streams = 2 * int(n_antennas)
    M = N // (2 * int(n_channels)) if N > 0 else 0
    return {"raw": streams * (N * 5 // 4), "delays": streams * M, "phases": streams * M,
            "gains": streams * int(n_channels) * 2, "out": streams * N}


def check_sizes(n_antennas: int, n_channels: int, n_samples: int, **buffers):
    """Raise ValueError if any given buffer (raw, delays, phases, gains, out)
    is too small for a call of n_samples samples per polarization."""
    need = call_sizes(n_antennas, n_channels, n_samples)
    for name, t in buffers.items():
        if t is not None:
            _need(t, need["out" if name in ("out", "y_out", "g_out") else name], name)


class Stream:
    """One fe_stream: A antennas x 2 polarizations with state across calls.

    ``weights`` is a host float32 array of 2n*T taps (copied at creation).
    ``precision`` is "fp32" (default), "fp16" or "bf16" (the matrix-core
    variants of the FIR and FFT, FE_PREC_* in the header; above 8192 channels
    "fp16" means FP16 storage around the float32 two-level FFT, and "bf16"
    is refused).  ``path`` is "auto" (default), "split", "split_folded",
    "fused" or "matrix_fir" (fe_stream_set_schedule).
    Work is enqueued on ``hip_stream`` (default: torch's current stream).
    """

    def __init__(self, n_channels: int, taps: int, n_antennas: int, weights,
                 max_samples: int, spectra_per_heap: int = 256, max_delay: int = 128,
                 hip_stream=None, precision="fp32", path="auto"):
        import numpy as np
        L = load_library()
        w = np.ascontiguousarray(weights, dtype=np.float32)
        if w.size != 2 * n_channels * taps:
            raise ValueError("weights must hold 2*n*T values")
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self._w = w
        cfg = _Config(n_channels, taps, n_antennas, spectra_per_heap, max_delay, prec, max_samples,
                      w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
        h = _vp()
        _check(L.fe_stream_create(ctypes.byref(cfg), _hip_stream(hip_stream), ctypes.byref(h)),
               "fe_stream_create")
        self._h = h
        if path != "auto":
            self.set_schedule(path, 0)
        self.n, self.taps, self.A = n_channels, taps, n_antennas
        self.precision = prec
        self.S, self.max_delay, self.max_samples = spectra_per_heap, max_delay, max_samples

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            _check(load_library().fe_stream_destroy(self._h), "fe_stream_destroy")
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

    # -- calls ------------------------------------------------------------
    def set_hip_stream(self, stream):
        _check(load_library().fe_stream_set_hip_stream(self._h, _hip_stream(stream)),
               "fe_stream_set_hip_stream")

    def reset(self):
        _check(load_library().fe_stream_reset(self._h), "fe_stream_reset")

    def status(self) -> int:
        """Synchronize and return the sticky status (FE_OK or FE_EDELAY)."""
        st = int(load_library().fe_stream_status(self._h))
        if st not in (FE_OK, FE_EDELAY):
            raise FEngineError(st, "fe_stream_status")
        return st

    def timing(self, enable: bool):
        """Record HIP events around this stream's kernels on every call."""
        _check(load_library().fe_stream_timing(self._h, 1 if enable else 0), "fe_stream_timing")

    def timing_read(self):
        """(fir_ms, post_ms, turn_ms, calls) summed since the last read; synchronizes."""
        a, b, t, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), _i64()
        _check(load_library().fe_stream_timing_read(self._h, ctypes.byref(a), ctypes.byref(b),
                                                    ctypes.byref(t), ctypes.byref(c)),
               "fe_stream_timing_read")
        return a.value, b.value, t.value, int(c.value)

    def _args(self, raw, n_samples, delays, phases=None, gains=None):
        import torch
        check_sizes(self.A, self.n, n_samples, raw=raw, delays=delays, phases=phases, gains=gains)
        out = [self._h, _ptr(raw, torch.uint8, "raw"), int(n_samples), _ptr(delays, torch.float64, "delays")]
        if phases is not None:
            out.append(_ptr(phases, torch.float64, "phases"))
        if gains is not None:
            out.append(_ptr(gains, torch.float32, "gains"))
        return out

    def channelize(self, raw, n_samples: int, delays, phases, gains, out):
        """Enqueue fe_channelize; ``out`` int8 [A][M/S_h][n][S_h][2][2]."""
        import torch
        a = self._args(raw, n_samples, delays, phases, gains) + [_ptr(out, torch.int8, "out")]
        check_sizes(self.A, self.n, n_samples, out=out)
        _check(load_library().fe_channelize(*a), "fe_channelize")

    def channelize_noalloc(self, raw, n_samples: int, delays, phases, gains, out):
        """Enqueue fe_channelize_noalloc (the call's intermediate buffers in the
        library's static device scratch; see the header for its limit)."""
        import torch
        a = self._args(raw, n_samples, delays, phases, gains) + [_ptr(out, torch.int8, "out")]
        check_sizes(self.A, self.n, n_samples, out=out)
        _check(load_library().fe_channelize_noalloc(*a), "fe_channelize_noalloc")

    def channelize_prequant(self, raw, n_samples: int, delays, phases, gains, y_out):
        """Enqueue fe_channelize_prequant; ``y_out`` float32 [A][2][M][n][2]."""
        import torch
        a = self._args(raw, n_samples, delays, phases, gains) + [_ptr(y_out, torch.float32, "y_out")]
        check_sizes(self.A, self.n, n_samples, y_out=y_out)
        _check(load_library().fe_channelize_prequant(*a), "fe_channelize_prequant")

    def channelize_fir(self, raw, n_samples: int, delays, g_out):
        """Enqueue fe_channelize_fir; ``g_out`` float32 [A][2][M][2n]."""
        import torch
        a = self._args(raw, n_samples, delays) + [_ptr(g_out, torch.float32, "g_out")]
        check_sizes(self.A, self.n, n_samples, g_out=g_out)
        _check(load_library().fe_channelize_fir(*a), "fe_channelize_fir")


    def autotune(self, raw, n_samples: int, delays, phases, gains, out, iters: int = 3) -> int:
        """fe_stream_autotune on these buffers; returns the chosen FIR run
        length (0 = per-launch default).  Resets the stream."""
        import torch
        a = self._args(raw, n_samples, delays, phases, gains) + [_ptr(out, torch.int8, "out")]
        check_sizes(self.A, self.n, n_samples, out=out)
        choice = ctypes.c_int()
        _check(load_library().fe_stream_autotune(*a, int(iters), ctypes.byref(choice)),
               "fe_stream_autotune")
        return int(choice.value)

    def set_tuning(self, fir_batches: int):
        _check(load_library().fe_stream_set_tuning(self._h, int(fir_batches)), "fe_stream_set_tuning")

    def set_fft_parts(self, parts: int):
        """fe_stream_set_fft_parts (above 8192 channels; 0 = per call)."""
        _check(load_library().fe_stream_set_fft_parts(self._h, int(parts)), "fe_stream_set_fft_parts")

    def fft_parts(self) -> int:
        p = ctypes.c_int()
        _check(load_library().fe_stream_get_fft_parts(self._h, ctypes.byref(p)), "fe_stream_get_fft_parts")
        return int(p.value)

    def set_schedule(self, path, fir_batches: int = 0):
        """fe_stream_set_schedule; ``path`` "auto", "split", "fused" or FE_PATH_*."""
        p = PATHS[path] if isinstance(path, str) else int(path)
        _check(load_library().fe_stream_set_schedule(self._h, p, int(fir_batches)), "fe_stream_set_schedule")

    def schedule(self):
        """(path that runs: "split", "fused" or "matrix_fir", fir_batches)."""
        p, b = ctypes.c_int(), ctypes.c_int()
        _check(load_library().fe_stream_get_schedule(self._h, ctypes.byref(p), ctypes.byref(b)),
               "fe_stream_get_schedule")
        names = {FE_PATH_FUSED: "fused", FE_PATH_MATRIX_FIR: "matrix_fir", FE_PATH_SPLIT_FOLDED: "split_folded"}
        return names.get(p.value, "split"), int(b.value)

    def _call(self, raw, n_samples, delays, phases, gains, out) -> _Call:
        import torch
        a = self._args(raw, n_samples, delays, phases, gains)
        o = _ptr(out, torch.int8, "out")
        check_sizes(self.A, self.n, n_samples, out=out)
        return _Call(a[1].value, int(n_samples), a[3].value, a[4].value, a[5].value, o.value)


class Batch:
    """fe_batch: one call of every member stream as a unit, run eagerly
    (``run``) or captured once into a HIP graph (``capture``) and replayed
    with one graph launch (``launch``).  ``calls[i]`` is the tuple
    (raw, n_samples, delays, phases, gains, out) of member i."""

    def __init__(self, members, hip_stream=None):
        L = load_library()
        self.members = list(members)
        arr = (_vp * len(self.members))(*[m._h for m in self.members])
        h = _vp()
        _check(L.fe_batch_create(arr, len(self.members), _hip_stream(hip_stream), ctypes.byref(h)),
               "fe_batch_create")
        self._h = h
        self._keep = None

    def _calls(self, calls):
        if len(calls) != len(self.members):
            raise ValueError("one call per member")
        arr = (_Call * len(calls))(*[m._call(*c) for m, c in zip(self.members, calls)])
        return arr

    def run(self, calls):
        arr = self._calls(calls)
        _check(load_library().fe_batch_run(self._h, arr), "fe_batch_run")

    def capture(self, calls):
        arr = self._calls(calls)
        self._keep = list(calls)            # the graph refers to these buffers
        _check(load_library().fe_batch_capture(self._h, arr), "fe_batch_capture")

    def launch(self):
        _check(load_library().fe_batch_launch(self._h), "fe_batch_launch")

    def set_grouped(self, grouped: bool):
        """fe_batch_set_grouped: grouped launches, or every member on its own fork stream (default)."""
        _check(load_library().fe_batch_set_grouped(self._h, 1 if grouped else 0), "fe_batch_set_grouped")

    def close(self):
        if getattr(self, "_h", None):
            _check(load_library().fe_batch_destroy(self._h), "fe_batch_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_unpack10(raw, first: int, count: int, out, hip_stream=None):
    """Enqueue fe_debug_unpack10 (int32 ``out`` of ``count`` samples)."""
    import torch
    _check(load_library().fe_debug_unpack10(_ptr(raw, torch.uint8, "raw"), int(first), int(count),
                                            _ptr(out, torch.int32, "out"), _hip_stream(hip_stream)),
           "fe_debug_unpack10")
