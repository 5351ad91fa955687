"""Parity criteria between the HIP path and the FP64 oracle.

TEST INFRASTRUCTURE ONLY (used by the tests, the smoke check and nothing in
the product path).

* pre-quantisation spectra (float32 path): per spectrum the normwise
  relative error ||Y - Y_ref|| / ||Y_ref|| <= 1e-5, and elementwise
  |Y_k - Y_ref,k| <= 1e-5 * max(|Y_ref,k|, rms of Y_ref over the spectrum);
  an all-zero reference spectrum must be exactly zero;
* int8 output: equal, except where the oracle's value lies within 1e-3 of a
  rounding boundary (a half-integer), where |q - q_ref| <= 1.
"""
from __future__ import annotations

import numpy as np

PREQUANT_RTOL = 1e-5
BOUNDARY_BAND = 1e-3


def prequant_errors(y, y_ref):
    """Return (worst normwise error, worst elementwise ratio) over spectra.

    ``y`` and ``y_ref`` are complex arrays [..., n]; the last axis is one
    spectrum.  Raises AssertionError on an all-zero reference spectrum whose
    counterpart is not exactly zero.
    """
    y = np.asarray(y, dtype=np.complex128)
    y_ref = np.asarray(y_ref, dtype=np.complex128)
    assert y.shape == y_ref.shape, (y.shape, y_ref.shape)
    d = np.abs(y - y_ref)
    mag = np.abs(y_ref)
    norm = np.sqrt(np.sum(mag ** 2, axis=-1))
    zero = norm == 0
    if zero.any():
        assert not np.abs(y[zero]).any(), "zero reference spectrum with non-zero output"
    nz = ~zero
    if not nz.any():
        return 0.0, 0.0
    normwise = np.sqrt(np.sum(d ** 2, axis=-1))[nz] / norm[nz]
    rms = norm / np.sqrt(y_ref.shape[-1])
    scale = np.maximum(mag, rms[..., None])
    elem = (d / np.where(scale > 0, scale, 1.0))[nz]
    return float(normwise.max()), float(elem.max())


def assert_prequant_close(y, y_ref, rtol: float = PREQUANT_RTOL):
    nw, el = prequant_errors(y, y_ref)
    assert nw <= rtol, "normwise relative error %.3g > %.3g" % (nw, rtol)
    assert el <= rtol, "elementwise scaled error %.3g > %.3g" % (el, rtol)
    return nw, el


def near_boundary(v, band: float = BOUNDARY_BAND):
    """True where float value v is within ``band`` of a half-integer."""
    v = np.asarray(v, dtype=np.float64)
    return np.abs(np.abs(v - np.floor(v)) - 0.5) < band


def int8_mismatches(q, q_ref, v_ref, band: float = BOUNDARY_BAND):
    """Count (hard mismatches, tolerated boundary differences).

    ``q``, ``q_ref`` int8 arrays of equal shape; ``v_ref`` the oracle's real
    values (same shape) that q_ref quantises.
    """
    q = np.asarray(q, dtype=np.int16)
    q_ref = np.asarray(q_ref, dtype=np.int16)
    assert q.shape == q_ref.shape == np.shape(v_ref)
    diff = q != q_ref
    nb = near_boundary(v_ref, band)
    hard = diff & ~(nb & (np.abs(q - q_ref) <= 1))
    return int(hard.sum()), int((diff & ~hard).sum())


def heap_values(y_plain, S: int):
    """Oracle values y [A][2][M][n] (complex) in heap order
    [A][M/S][n][S][2][2] (re, im), matching the int8 output layout."""
    y_plain = np.asarray(y_plain)
    A, P, M, n = y_plain.shape
    t = y_plain.reshape(A, P, M // S, S, n).transpose(0, 2, 4, 3, 1)
    return np.stack([t.real, t.imag], axis=-1)
