"""Host-only checks of the C ABI: the library loads, exports every function
declared in include/fengine.h, and rejects bad arguments on the host before
touching a device.  No kernel runs here."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2303_09886_amd as fe
from paper_2303_09886_amd import build as fe_build
from paper_2303_09886_amd.fengine import _Config, load_library

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if fe_build.needs_build():
        fe_build.build()
    return load_library()


def _declared_functions():
    names = set()
    for hdr in os.listdir(os.path.join(ROOT, "include")):
        if hdr.endswith(".h"):
            text = open(os.path.join(ROOT, "include", hdr)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(fe_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert "fe_channelize" in names and len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name


def test_version_and_strerror(lib):
    assert fe.version() == 200
    for code in (fe.FE_OK, fe.FE_EINVAL, fe.FE_ENOMEM, fe.FE_EHIP, fe.FE_EDELAY, fe.FE_ESIZE):
        assert lib.fe_strerror(code)
    assert lib.fe_strerror(-99) == b"unknown status"


def _cfg(**kw):
    w = np.zeros(2 * kw.get("n_channels", 1024) * kw.get("taps", 16), dtype=np.float32)
    base = dict(n_channels=1024, taps=16, n_antennas=1, spectra_per_heap=256, max_delay=128,
                precision=0, max_samples=1 << 20)
    base.update(kw)
    c = _Config(base["n_channels"], base["taps"], base["n_antennas"], base["spectra_per_heap"],
                base["max_delay"], base["precision"], base["max_samples"],
                w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    return c, w


@pytest.mark.parametrize("bad", [
    dict(n_channels=1000), dict(n_channels=128), dict(n_channels=16384), dict(taps=0),
    dict(taps=33), dict(n_antennas=0), dict(spectra_per_heap=0), dict(max_delay=-1),
    dict(max_samples=0), dict(max_samples=(1 << 20) + 2048), dict(max_samples=1 << 29),
    dict(precision=3), dict(precision=-1),
])
def test_create_rejects_bad_config(lib, bad):
    cfg, _w = _cfg(**bad)
    h = ctypes.c_void_p()
    assert lib.fe_stream_create(ctypes.byref(cfg), None, ctypes.byref(h)) == fe.FE_EINVAL
    assert not h.value


def test_fp16_stream_rejects_non_finite_taps(lib):
    cfg, w = _cfg(precision=fe.FE_PREC_FP16)
    w[7] = np.inf
    h = ctypes.c_void_p()
    assert lib.fe_stream_create(ctypes.byref(cfg), None, ctypes.byref(h)) == fe.FE_EINVAL
    assert not h.value


def test_null_arguments_are_rejected(lib):
    h = ctypes.c_void_p()
    assert lib.fe_stream_create(None, None, ctypes.byref(h)) == fe.FE_EINVAL
    cfg, _w = _cfg()
    cfg.weights = ctypes.POINTER(ctypes.c_float)()
    assert lib.fe_stream_create(ctypes.byref(cfg), None, ctypes.byref(h)) == fe.FE_EINVAL
    dummy = ctypes.c_void_p(0x1000)
    assert lib.fe_channelize(None, dummy, 1 << 20, dummy, dummy, dummy, dummy) == fe.FE_EINVAL
    assert lib.fe_channelize_prequant(None, dummy, 1 << 20, dummy, dummy, dummy, dummy) == fe.FE_EINVAL
    assert lib.fe_channelize_fir(None, dummy, 1 << 20, dummy, dummy) == fe.FE_EINVAL
    assert lib.fe_stream_reset(None) == fe.FE_EINVAL
    assert lib.fe_stream_status(None) == fe.FE_EINVAL
    assert lib.fe_stream_set_hip_stream(None, None) == fe.FE_EINVAL
    assert lib.fe_stream_destroy(None) == fe.FE_OK
    assert lib.fe_debug_unpack10(None, 0, 4, dummy, None) == fe.FE_EINVAL
    assert lib.fe_debug_unpack10(dummy, -1, 4, dummy, None) == fe.FE_EINVAL
    assert lib.fe_debug_unpack10(dummy, 0, 0, dummy, None) == fe.FE_OK


def test_batch_and_tuning_reject_bad_arguments(lib):
    from paper_2303_09886_amd import fengine
    h = ctypes.c_void_p()
    assert lib.fe_batch_create(None, 1, None, ctypes.byref(h)) == fe.FE_EINVAL
    arr = (ctypes.c_void_p * 1)(None)
    assert lib.fe_batch_create(arr, 1, None, ctypes.byref(h)) == fe.FE_EINVAL
    assert lib.fe_batch_create(arr, 0, None, ctypes.byref(h)) == fe.FE_EINVAL
    assert not h.value
    assert lib.fe_batch_launch(None) == fe.FE_EINVAL
    assert lib.fe_batch_run(None, None) == fe.FE_EINVAL
    assert lib.fe_batch_capture(None, None) == fe.FE_EINVAL
    assert lib.fe_batch_destroy(None) == fe.FE_OK
    assert lib.fe_batch_set_grouped(None, 1) == fe.FE_EINVAL
    dummy = ctypes.c_void_p(0x1000)
    assert lib.fe_stream_autotune(None, dummy, 1 << 20, dummy, dummy, dummy, dummy, 1, None) == fe.FE_EINVAL
    assert lib.fe_stream_set_tuning(None, 1) == fe.FE_EINVAL
    assert lib.fe_stream_set_schedule(None, fe.FE_PATH_FUSED, 0) == fe.FE_EINVAL
    assert lib.fe_stream_get_schedule(None, None, None) == fe.FE_EINVAL
    assert ctypes.sizeof(fengine._Call) == 48


def test_binding_refuses_host_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(TypeError):
        fe.debug_unpack10(torch.zeros(8, dtype=torch.uint8), 0, 4, torch.zeros(4, dtype=torch.int32))


def test_missing_library_fails_loudly(tmp_path):
    from paper_2303_09886_amd import fengine
    saved = fengine._lib
    try:
        fengine._lib = None
        with pytest.raises(fe.FEngineError):
            load_library(str(tmp_path / "nope.so"))
    finally:
        fengine._lib = saved


def test_binding_refuses_undersized_buffers():
    """The binding checks every buffer against the header's layout before any
    call (an undersized buffer would be read or written past its end)."""
    import torch
    from paper_2303_09886_amd.fengine import call_sizes, check_sizes
    A, n, N = 2, 256, 2 * 256 * 8
    need = call_sizes(A, n, N)
    assert need == {"raw": 4 * N * 5 // 4, "delays": 4 * 8, "phases": 4 * 8, "gains": 4 * n * 2,
                    "out": 4 * N}
    ok = {"raw": torch.empty(need["raw"], dtype=torch.uint8),
          "delays": torch.empty(need["delays"], dtype=torch.float64),
          "phases": torch.empty(need["phases"], dtype=torch.float64),
          "gains": torch.empty(need["gains"], dtype=torch.float32),
          "out": torch.empty(need["out"], dtype=torch.int8)}
    check_sizes(A, n, N, **ok)
    check_sizes(A, n, N, y_out=torch.empty(4 * N, dtype=torch.float32),
                g_out=torch.empty(4 * N, dtype=torch.float32))
    for name in ok:
        small = dict(ok)
        small[name] = ok[name][:-1]
        with pytest.raises(ValueError, match=name):
            check_sizes(A, n, N, **small)
    for name in ("y_out", "g_out"):
        with pytest.raises(ValueError, match=name):
            check_sizes(A, n, N, **{name: torch.empty(4 * N - 1, dtype=torch.float32)})
    # a call twice as long needs twice the buffers
    with pytest.raises(ValueError):
        check_sizes(A, n, 2 * N, **ok)
