"""Seeded synthetic inputs for the F-engine channelizer.

This module only *produces inputs*: digitizer samples (Gaussian noise plus
tones, clipped to the signed 10-bit range), their packed 10-bit byte stream,
per-spectrum delays and phases, per-channel complex gains and the PFB
prototype filter.  It performs no step of the channelizer itself, so the
oracle and the HIP path can both consume its arrays without sharing any of
the method's arithmetic.

Input format (Sec. 2.1 step 1 and Sec. 2.2 of the paper: signed 10-bit
samples, packed, one polarization per stream): each sample is a 10-bit two's
complement code; codes are concatenated into a bitstream most-significant bit
first, and the bitstream is cut into bytes most-significant bit first.  Four
samples therefore occupy exactly five bytes.

Workload recipe (the paper uses live or simulated digitizers; there is no
public dataset):

* samples  x_i = clip(rint(sigma*N(0,1) + sum_q A_q cos(2*pi*f_q*i + psi_q)),
  -511, 511), sigma = 30, three tones common to both polarizations of an
  antenna, independent noise per polarization, tone 1 centred on channel
  ``tone_channel`` (the paper's precision study puts a tone in channel 192 of
  1024), the other two at U(0.01, 0.49) cycles/sample, A_q ~ U(10, 100),
  psi_q ~ U(0, 2*pi);
* delays   d_F = d0 + r * 2n * F (+ a small per-polarization offset),
  d0 ~ U(5, 95), r ~ U(-r_max, r_max) with r_max the workload's rate capped so
  that d stays within [1, 127] over the whole stream;
* phases   phi_F = phi0 + w * 2n * F, phi0 ~ U(0, 2*pi), w ~ U(-1e-4, 1e-4);
* gains    |G| ~ U(0.5, 2), arg G ~ U(0, 2*pi), per (antenna, pol, channel);
* taps     Hann-windowed sinc (Sec. 5.2), see :func:`pfb_taps`.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

__all__ = [
    "Shape", "SMALL", "LARGE", "BATCH16", "STREAM32K", "pfb_taps", "pack10", "samples10",
    "Workload", "make_workload", "heap_count",
]


@dataclasses.dataclass(frozen=True)
class Shape:
    """One channelizer configuration.

    n         channels (the PFB computes a 2n-point real FFT)
    taps      PFB taps T
    antennas  A; every antenna has two polarizations
    samples   N, samples per polarization handed over in one call
    spectra_per_heap  S_h, spectra per output heap (256 in the paper, Sec. 2.2)
    max_delay D_max, the largest integer (coarse) delay the stream accepts
    """
    n: int
    taps: int
    antennas: int
    samples: int
    spectra_per_heap: int = 256
    max_delay: int = 128

    @property
    def spectra(self) -> int:
        return self.samples // (2 * self.n)


#: Small configuration: one antenna, 2^20 samples/pol, 1024 channels, 16 taps.
SMALL = Shape(n=1024, taps=16, antennas=1, samples=1 << 20)
#: MeerKAT-like scale: four antennas, 2^24 samples/pol, 4096 channels, 16 taps.
LARGE = Shape(n=4096, taps=16, antennas=4, samples=1 << 24)
#: Batched workload: 16 single-antenna streams of uneven shape -- channels
#: 1024 / 4096 / 8192 / 32768, taps 8 / 16 / 24, 2^22 .. 2^24 samples/pol per
#: call, heaps of 64 spectra.
BATCH16 = tuple(
    Shape(n=n, taps=t, antennas=1, samples=1 << lg, spectra_per_heap=64)
    for n, t, lg in [
        (1024, 8, 22), (4096, 16, 23), (8192, 24, 24), (32768, 16, 24),
        (1024, 16, 23), (4096, 24, 24), (8192, 8, 22), (32768, 8, 22),
        (1024, 24, 24), (4096, 8, 22), (8192, 16, 23), (32768, 24, 23),
        (1024, 16, 22), (4096, 16, 24), (8192, 16, 24), (32768, 16, 22),
    ])
#: Streaming service: one wide-band antenna, 32768 channels, 16 taps; chunks
#: are whole numbers of 2^20 samples (32 spectra), heaps of 16 spectra.
STREAM32K = Shape(n=32768, taps=16, antennas=1, samples=1 << 20, spectra_per_heap=16)


def heap_count(shape: Shape) -> int:
    return shape.spectra // shape.spectra_per_heap


def pfb_taps(n: int, taps: int) -> np.ndarray:
    """Hann-windowed sinc prototype filter, float32[2n*taps].

    h[u] = hann(u) * sinc((u - (L-1)/2) / (2n)), L = 2n*taps, with the
    symmetric Hann window of length L; the sinc's first nulls sit one channel
    width (2n samples) either side of the centre.  Normalised so that
    sum(h^2) = 1 (white noise keeps its variance through the filter bank).
    Computed in float64 and rounded once to float32; the float32 array is the
    canonical input to every implementation.
    """
    L = 2 * n * taps
    u = np.arange(L, dtype=np.float64)
    h = np.hanning(L) * np.sinc((u - (L - 1) / 2.0) / (2.0 * n))
    h /= np.sqrt(np.sum(h * h))
    return h.astype(np.float32)


def pack10(x: np.ndarray) -> np.ndarray:
    """Pack signed 10-bit samples along the last axis into the byte stream.

    ``x`` holds integers in [-512, 511]; its last axis must be a multiple of
    4.  Returns uint8 with last axis 5/4 as long.  Sample bits go out MSB
    first, bytes are filled MSB first.
    """
    x = np.asarray(x)
    if x.shape[-1] % 4:
        raise ValueError("sample count must be a multiple of 4")
    if x.size and (x.min() < -512 or x.max() > 511):
        raise ValueError("samples outside the signed 10-bit range")
    code = (x.astype(np.int32) & 0x3FF).astype(np.uint32)
    q = code.reshape(*x.shape[:-1], x.shape[-1] // 4, 4)
    c0, c1, c2, c3 = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    out = np.empty(q.shape[:-1] + (5,), dtype=np.uint8)
    out[..., 0] = c0 >> 2
    out[..., 1] = ((c0 & 0x3) << 6) | (c1 >> 4)
    out[..., 2] = ((c1 & 0xF) << 4) | (c2 >> 6)
    out[..., 3] = ((c2 & 0x3F) << 2) | (c3 >> 8)
    out[..., 4] = c3 & 0xFF
    return out.reshape(*x.shape[:-1], x.shape[-1] * 5 // 4)


def _tone_sum(count: int, tones, start: int = 0) -> np.ndarray:
    """sum_q A_q cos(2*pi*f_q*i + psi_q) for i in [start, start+count).

    Evaluated blockwise with the angle-addition identity so that only
    O(count/B + B) cosines are taken; all in float64.
    """
    B = 4096
    nb = -(-count // B)
    off = np.arange(B, dtype=np.float64)
    base = start + B * np.arange(nb, dtype=np.float64)
    acc = np.zeros((nb, B), dtype=np.float64)
    for f, amp, psi in tones:
        a = 2.0 * np.pi * np.mod(f * base, 1.0) + psi
        b = 2.0 * np.pi * np.mod(f * off, 1.0)
        ca, sa = amp * np.cos(a), amp * np.sin(a)
        acc += np.multiply.outer(ca, np.cos(b))
        acc -= np.multiply.outer(sa, np.sin(b))
    return acc.reshape(-1)[:count]


def samples10(rng: np.random.Generator, count: int, sigma: float, tones,
              start: int = 0, tone_sum: Optional[np.ndarray] = None) -> np.ndarray:
    """int16 samples: clip(rint(sigma*N(0,1) + tones), -511, 511)."""
    if tone_sum is None:
        tone_sum = _tone_sum(count, tones, start)
    v = sigma * rng.standard_normal(count) + tone_sum
    return np.clip(np.rint(v), -511, 511).astype(np.int16)


@dataclasses.dataclass
class Workload:
    """All inputs of a stream of ``total`` samples per polarization.

    x       int16 [A][2][total]            the samples (for reference only)
    raw     uint8 [A][2][total*5/4]        packed 10-bit byte stream
    delays  float64 [A][2][total/(2n)]     total delay d_F of spectrum F, in samples
    phases  float64 [A][2][total/(2n)]     phase phi_F of spectrum F, radians
    gains   float32 [A][2][n][2]           complex gain per channel (re, im)
    weights float32 [2n*T]                 PFB prototype filter h
    """
    shape: Shape
    total: int
    x: np.ndarray
    raw: np.ndarray
    delays: np.ndarray
    phases: np.ndarray
    gains: np.ndarray
    weights: np.ndarray

    def chunk(self, start: int, count: int):
        """Inputs of one call covering samples [start, start+count)."""
        n2 = 2 * self.shape.n
        if start % n2 or count % n2:
            raise ValueError("chunk bounds must be whole spectra")
        f0, f1 = start // n2, (start + count) // n2
        b0, b1 = start * 5 // 4, (start + count) * 5 // 4
        return (np.ascontiguousarray(self.raw[:, :, b0:b1]),
                np.ascontiguousarray(self.delays[:, :, f0:f1]),
                np.ascontiguousarray(self.phases[:, :, f0:f1]))


def make_workload(shape: Shape, seed: int, total: Optional[int] = None, *,
                  sigma: float = 30.0, delay_rate: float = 1e-5,
                  pol_delay_offset: float = 0.1, tone_channel: Optional[int] = None,
                  antennas: Optional[int] = None) -> Workload:
    """Build the seeded inputs of ``shape`` for ``total`` samples per pol.

    ``delay_rate`` is the largest delay slope in samples per sample; the
    default (1e-5) is far above the paper's sidereal rate (< 3e-9, Sec. 3.3)
    so that the integer part of the delay steps inside one call.
    """
    n, A = shape.n, (shape.antennas if antennas is None else antennas)
    total = shape.samples if total is None else total
    if total % (2 * n):
        raise ValueError("total must be a whole number of spectra")
    M = total // (2 * n)
    if tone_channel is None:
        tone_channel = 192 * n // 1024
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(A + 3)
    x = np.empty((A, 2, total), dtype=np.int16)
    for a in range(A):
        r_tone, r_n0, r_n1 = [np.random.default_rng(k) for k in kids[a].spawn(3)]
        tones = [(tone_channel / (2.0 * n), r_tone.uniform(10, 100),
                  r_tone.uniform(0, 2 * np.pi))]
        for _ in range(2):
            tones.append((r_tone.uniform(0.01, 0.49), r_tone.uniform(10, 100),
                          r_tone.uniform(0, 2 * np.pi)))
        ts = _tone_sum(total, tones)
        x[a, 0] = samples10(r_n0, total, sigma, tones, tone_sum=ts)
        x[a, 1] = samples10(r_n1, total, sigma, tones, tone_sum=ts)
        del ts
    raw = pack10(x)

    rd = np.random.default_rng(kids[A])
    F = np.arange(M, dtype=np.float64)
    delays = np.empty((A, 2, M), dtype=np.float64)
    span = 2.0 * n * max(M - 1, 1)
    for a in range(A):
        d0 = rd.uniform(5, 95)
        # the slope is capped so that d stays in [1, 127] over the stream
        r_max = min(delay_rate, (d0 - 1.0) / span, (127.0 - d0) / span)
        rate = rd.uniform(-r_max, r_max)
        off = rd.uniform(-pol_delay_offset, pol_delay_offset)
        delays[a, 0] = d0 + rate * 2 * n * F
        delays[a, 1] = d0 + off + rate * 2 * n * F

    rp = np.random.default_rng(kids[A + 1])
    phases = np.empty((A, 2, M), dtype=np.float64)
    for a in range(A):
        for p in range(2):
            phases[a, p] = rp.uniform(0, 2 * np.pi) + rp.uniform(-1e-4, 1e-4) * 2 * n * F

    rg = np.random.default_rng(kids[A + 2])
    mag = rg.uniform(0.5, 2.0, size=(A, 2, n))
    arg = rg.uniform(0, 2 * np.pi, size=(A, 2, n))
    gains = np.stack([mag * np.cos(arg), mag * np.sin(arg)], axis=-1).astype(np.float32)

    return Workload(shape=dataclasses.replace(shape, antennas=A), total=total, x=x,
                    raw=raw, delays=delays, phases=phases, gains=gains,
                    weights=pfb_taps(n, shape.taps))
