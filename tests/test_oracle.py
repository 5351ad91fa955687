"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test ties one oracle step to something other than the oracle itself:
a worked example, a brute-force computation, a closed form, an invariant or
a textbook routine.  The mistakes each is meant to catch are named in its
docstring.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth


# --------------------------------------------------------------------------
# Step 1 -- unpacking (Sec. 2.1 item 1, Sec. 2.2)
# --------------------------------------------------------------------------

def _read_golden(path):
    rows = {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = line.split(":", 1)
        rows[k.strip()] = v.split()
    return rows


def test_unpack_worked_example(golden_dir):
    """Hand-derived bytes of [1, -1, -512, 511]: catches bit order and sign errors."""
    g = _read_golden(os.path.join(golden_dir, "unpack10_example.txt"))
    samples = [int(v) for v in g["samples"]]
    raw = bytes(int(b, 16) for b in g["bytes"])
    assert list(oracle.unpack10(raw)) == samples
    assert synth.pack10(np.array(samples)).tobytes() == raw


def _packbits_reference(x):
    """Independent packer built on numpy.packbits (bit arrays, MSB first)."""
    code = (np.asarray(x, dtype=np.int64) & 0x3FF)
    bits = ((code[:, None] >> np.arange(9, -1, -1)[None, :]) & 1).astype(np.uint8)
    return np.packbits(bits.reshape(-1))


def test_unpack_all_codes_all_phases():
    """Every 10-bit code at each of the four bit phases (10*i mod 8)."""
    codes = np.arange(-512, 512)
    for lead in range(4):                        # shifts the bit phase of every code
        x = np.concatenate([np.full(lead, 77), codes, np.full((4 - (lead + 1024) % 4) % 4, -3)])
        raw = _packbits_reference(x)
        got = oracle.unpack10(raw, 0, x.size)
        assert np.array_equal(got, x)
        assert np.array_equal(synth.pack10(x), raw)


def test_unpack_offset_reads():
    """Reading from a non-zero first sample: catches off-by-one byte offsets."""
    x = np.random.default_rng(3).integers(-512, 512, size=4000)
    raw = _packbits_reference(x)
    for first in (0, 1, 2, 3, 5, 17, 999):
        assert np.array_equal(oracle.unpack10(raw, first, 100), x[first:first + 100])


# --------------------------------------------------------------------------
# Steps 2/4 -- delay split (Sec. 2.1 items 2 and 4, Sec. 3.3)
# --------------------------------------------------------------------------

def test_delay_split_table(golden_dir):
    for line in open(os.path.join(golden_dir, "delay_split.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        d, valid, c, tau = line.split()
        ok, cc, tt = oracle.split_delay(float(d), 128)
        assert (ok, cc) == (bool(int(valid)), int(c)), line
        assert tt == float(tau), line


def test_delay_split_properties():
    """c + tau reproduces d exactly and tau lies in [-0.5, 0.5)."""
    rng = np.random.default_rng(5)
    for d in np.concatenate([rng.uniform(-0.5, 128.4, 2000), np.arange(0, 128) + 0.5,
                             np.nextafter(np.arange(0, 128) + 0.5, -np.inf)]):
        ok, c, tau = oracle.split_delay(d, 128)
        assert ok
        assert -0.5 <= tau < 0.5
        assert c + tau == d                      # exact in float64


# --------------------------------------------------------------------------
# Step 3 -- Fourier transform
# --------------------------------------------------------------------------

def _dft_longdouble(x):
    """O(N^2) DFT in extended precision, angles reduced exactly in integers."""
    N = len(x)
    xr = np.asarray(np.real(x), dtype=np.longdouble)
    xi = np.asarray(np.imag(x), dtype=np.longdouble)
    t = np.arange(N)
    X = np.empty(N, dtype=np.complex128)
    two_pi = np.longdouble(2) * np.arccos(np.longdouble(-1))
    for k in range(N):
        m = (t * k) % N                          # exact reduction of t*k
        ang = -two_pi * m.astype(np.longdouble) / N
        c, s = np.cos(ang), np.sin(ang)
        X[k] = complex(np.sum(xr * c - xi * s), np.sum(xr * s + xi * c))
    return X


@pytest.mark.parametrize("N", [1, 2, 4, 8, 16, 32, 64, 128, 256])
def test_fft_against_brute_force(N):
    """Catches wrong sign of the exponent, bad bit reversal, bad twiddles."""
    rng = np.random.default_rng(N)
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    X = oracle.fft(x)
    ref = _dft_longdouble(x)
    assert np.max(np.abs(X - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(X - np.fft.fft(x))) <= 1e-12 * np.max(np.abs(ref))


def test_fft_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        oracle.fft(np.ones(12))


@pytest.mark.parametrize("n", [4, 32, 512])
def test_rfft_keep_parseval_and_bins(n):
    """Real 2n-point transform keeps k = 0..n-1: Parseval with a separately
    computed Nyquist bin catches a dropped or doubled bin and a wrong scale."""
    rng = np.random.default_rng(n)
    g = rng.standard_normal(2 * n)
    X = oracle.rfft_keep(g)
    assert X.shape == (n,)
    nyq = np.sum(g * (-1.0) ** np.arange(2 * n))
    lhs = np.sum(g * g)
    rhs = (X[0].real ** 2 + 2 * np.sum(np.abs(X[1:]) ** 2) + nyq ** 2) / (2 * n)
    assert abs(lhs - rhs) <= 1e-12 * lhs
    assert abs(X[0].imag) <= 1e-12 * np.abs(X).max()
    if n <= 32:
        full = _dft_longdouble(g)
        assert np.max(np.abs(X - full[:n])) <= 1e-13 * np.abs(full).max()
        # Hermitian symmetry of a real input's spectrum
        assert np.max(np.abs(full[1:][::-1] - np.conj(full[1:]))) <= 1e-12 * np.abs(full).max()


# --------------------------------------------------------------------------
# Step 3 -- PFB FIR (Eq. 1) and the whole filter bank
# --------------------------------------------------------------------------

def _taps(n, T, seed=0):
    """Asymmetric random taps: orientation mistakes are visible with these."""
    return np.random.default_rng(seed).standard_normal(2 * n * T).astype(np.float32)


@pytest.mark.parametrize("n,T", [(8, 4), (16, 3), (64, 16)])
def test_impulse_response_is_the_taps(n, T):
    """An impulse at sample p seen through spectrum F gives
    X_F[k] = h[u] exp(-2 pi i k (u mod 2n) / 2n), u = p - window start.
    Catches transposed tap indexing (w_{t,j} vs h[t + 2nj]), a wrong window
    position and a wrong FFT sign."""
    h = _taps(n, T)
    F = T + 3
    W = 2 * n * (F - T + 1)                    # window start, coarse delay 0
    k = np.arange(n)
    for u in [0, 1, 2 * n - 1, 2 * n, 2 * n * T - 1, 5 * n + 3]:
        if u >= 2 * n * T:
            continue
        s = np.zeros(2 * n * (F + 1))
        s[W + u] = 1.0
        X = oracle.rfft_keep(oracle.pfb_fir(s, n, T, h, F, 0))
        expect = float(h[u]) * np.exp(-2j * np.pi * k * (u % (2 * n)) / (2 * n))
        assert np.max(np.abs(X - expect)) <= 1e-14 * max(1.0, abs(float(h[u]))) * np.log2(2 * n)


def _H(h, n, delta):
    """Response of the prototype filter at offset ``delta`` channels:
    sum_u h[u] exp(-2 pi i u delta / 2n), extended precision."""
    u = np.arange(h.size, dtype=np.longdouble)
    two_pi = np.longdouble(2) * np.arccos(np.longdouble(-1))
    ang = -two_pi * u * np.longdouble(delta) / (2 * n)
    hh = h.astype(np.longdouble)
    return complex(np.sum(hh * np.cos(ang)), np.sum(hh * np.sin(ang)))


@pytest.mark.parametrize("k0,frac", [(5, 0.0), (12, 0.0), (7, 0.37)])
def test_tone_closed_form(k0, frac):
    """A tone A cos(2 pi f i + psi), f = (k0 + frac)/(2n), gives
    X_F[k] = (A/2)(e^{i a} H(k - k0') + e^{-i a} H(k + k0')), a = 2 pi f W + psi.
    Catches FIR/FFT index slips, sign errors and a wrong window origin."""
    n, T = 64, 4
    h = synth.pfb_taps(n, T)
    kk = k0 + frac
    f = kk / (2 * n)
    A, psi = 37.0, 0.7
    F = T + 2
    W = 2 * n * (F - T + 1)
    i = np.arange(2 * n * (F + 1))
    s = A * np.cos(2 * np.pi * f * i + psi)
    X = oracle.rfft_keep(oracle.pfb_fir(s, n, T, h, F, 0))
    a = 2 * np.pi * f * W + psi
    expect = np.array([(A / 2) * (np.exp(1j * a) * _H(h, n, k - kk) + np.exp(-1j * a) * _H(h, n, k + kk))
                       for k in range(n)])
    scale = np.abs(expect).max()
    assert np.max(np.abs(X - expect)) <= 1e-12 * scale
    # the tone lands in its channel: peak at k0 with (A/2)*sum(h) when bin-centred
    if frac == 0.0:
        assert np.argmax(np.abs(X)) == k0
        assert abs(abs(X[k0]) - (A / 2) * float(np.sum(h.astype(np.float64)))) <= 1e-3 * scale


def _full_path(x, n, T, delays, phases, gains, h, max_delay=40):
    """oracle.channelize on integer samples x[A][2][N] (packed first)."""
    raw = synth.pack10(x)
    N = x.shape[-1]
    return oracle.channelize(raw, N, n, T, max_delay, h, delays, phases, gains,
                             want=("g", "x", "y", "q", "valid"))


def _small_inputs(seed, n=32, T=4, M=24, A=2):
    rng = np.random.default_rng(seed)
    x = np.clip(np.rint(rng.normal(0, 60, size=(A, 2, 2 * n * M))), -512, 511).astype(np.int64)
    delays = rng.uniform(0, 30, size=(A, 2, M))
    phases = rng.uniform(0, 2 * np.pi, size=(A, 2, M))
    gains = rng.uniform(0.5, 2, size=(A, 2, n, 2)).astype(np.float32)
    h = synth.pfb_taps(n, T)
    return x, delays, phases, gains, h


def test_integer_delay_is_a_pure_shift():
    """Coarse delay c equals feeding the stream shifted by c samples with
    zero delay, bit for bit (Sec. 3.3: coarse delay is an index adjustment).
    Catches a wrong sign of c in Eq. (1)."""
    n, T, M = 32, 4, 24
    x, _, phases, gains, h = _small_inputs(11, n, T, M, A=1)
    N = x.shape[-1]
    for c in (1, 3, 17, 40):
        d = np.full((1, 2, M), float(c))
        r1 = _full_path(x, n, T, d, phases, gains, h)
        xs = np.zeros_like(x)
        xs[..., c:] = x[..., :N - c]
        r0 = _full_path(xs, n, T, np.zeros((1, 2, M)), phases, gains, h)
        for key in ("g", "x", "y", "q"):
            assert np.array_equal(r1[key], r0[key]), (c, key)


def test_fine_delay_matches_an_analytic_delay():
    """A bin-centred tone processed with delay d = c + tau matches the same
    tone delayed analytically by d and processed with zero delay, at its bin,
    up to the conjugate image term |H(2 k0)|.  The opposite sign of the
    phase ramp misses by ~|1 - e^{2 pi i k0 tau / n}|."""
    n, T = 64, 8
    h = synth.pfb_taps(n, T)
    k0 = 11
    f = k0 / (2 * n)
    A, psi = 50.0, 0.3
    F = T + 4
    i = np.arange(2 * n * (F + 1), dtype=np.float64)
    image = abs(_H(h, n, 2 * k0)) / abs(_H(h, n, 0))
    worst_wrong = 0.0
    for d in (3.3, 7.5, 12.49, 20.8, 0.26):
        ok, c, tau = oracle.split_delay(d, 64)
        assert ok
        s = A * np.cos(2 * np.pi * f * i + psi)
        X = oracle.rfft_keep(oracle.pfb_fir(s, n, T, h, F, c))
        Y = oracle.fine_delay_gain(X, tau, 0.0, np.ones(n, dtype=np.complex64))
        sd = A * np.cos(2 * np.pi * f * (i - d) + psi)
        X0 = oracle.rfft_keep(oracle.pfb_fir(sd, n, T, h, F, 0))
        rel = abs(Y[k0] - X0[k0]) / abs(X0[k0])
        assert rel <= 2 * image + 1e-12, (d, rel)
        Yw = oracle.fine_delay_gain(X, -tau, 0.0, np.ones(n, dtype=np.complex64))
        worst_wrong = max(worst_wrong, abs(Yw[k0] - X0[k0]) / abs(X0[k0]))
    assert worst_wrong > 1e-2


def test_phase_and_gain_are_linear_rotations():
    """phi rotates every channel by e^{i phi}; the gain multiplies (Sec. 2.1
    items 4-5).  A conjugated gain or a dropped phase term fails this."""
    n = 16
    rng = np.random.default_rng(2)
    X = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    G = (rng.uniform(0.5, 2, n) * np.exp(1j * rng.uniform(0, 6.28, n))).astype(np.complex64)
    Y0 = oracle.fine_delay_gain(X, 0.0, 0.0, np.ones(n, dtype=np.complex64))
    assert np.max(np.abs(Y0 - X)) <= 1e-15 * np.abs(X).max()
    Yp = oracle.fine_delay_gain(X, 0.0, 1.1, np.ones(n, dtype=np.complex64))
    assert np.max(np.abs(Yp - np.exp(1.1j) * X)) <= 1e-14 * np.abs(X).max()
    Yg = oracle.fine_delay_gain(X, 0.0, 0.0, G)
    assert np.max(np.abs(Yg - G.astype(np.complex128) * X)) <= 1e-14 * np.abs(Yg).max()
    # the fine-delay ramp at channel k is exp(-i pi k tau / n): k = 0 untouched
    Yt = oracle.fine_delay_gain(X, 0.4, 0.0, np.ones(n, dtype=np.complex64))
    assert abs(Yt[0] - X[0]) <= 1e-15 * abs(X[0])


def test_linearity_and_polarization_independence():
    """Pols are processed independently (Sec. 2.1, after item 6) and the
    pre-quantisation path is linear in the samples."""
    n, T, M = 32, 4, 24
    x, delays, phases, gains, h = _small_inputs(21, n, T, M, A=1)
    r = _full_path(x, n, T, delays, phases, gains, h)
    x2 = x.copy()
    x2[0, 1] = np.random.default_rng(9).integers(-400, 400, size=x.shape[-1])
    r2 = _full_path(x2, n, T, delays, phases, gains, h)
    assert np.array_equal(r["y"][0, 0], r2["y"][0, 0])
    assert not np.array_equal(r["y"][0, 1], r2["y"][0, 1])
    # linearity: y(x + x') = y(x) + y(x') within rounding
    xa = np.clip(x // 2, -256, 255)
    xb = np.clip(x - xa, -256, 255)
    ra = _full_path(xa, n, T, delays, phases, gains, h)
    rb = _full_path(xb, n, T, delays, phases, gains, h)
    rs = _full_path(xa + xb, n, T, delays, phases, gains, h)
    assert np.max(np.abs(ra["y"] + rb["y"] - rs["y"])) <= 1e-10 * np.abs(rs["y"]).max()


def test_stream_start_is_zero_and_spectrum_ranges_compose():
    """Spectra near the stream start read zeros before sample 0; computing a
    range of spectra in two pieces equals computing it at once."""
    n, T, M = 32, 4, 24
    x, delays, phases, gains, h = _small_inputs(31, n, T, M, A=2)
    raw = synth.pack10(x)
    N = x.shape[-1]
    full = oracle.channelize(raw, N, n, T, 40, h, delays, phases, gains, want=("y", "q"))
    a = oracle.channelize(raw, N, n, T, 40, h, delays, phases, gains, 0, 10, want=("y", "q"))
    b = oracle.channelize(raw, N, n, T, 40, h, delays, phases, gains, 10, M, want=("y", "q"))
    assert np.array_equal(np.concatenate([a["y"], b["y"]], axis=2), full["y"])
    assert np.array_equal(np.concatenate([a["q"], b["q"]], axis=2), full["q"])
    # spectrum 0 with zero delay sees only samples [0, 2n): brute force it
    g0 = oracle.pfb_fir(x[0, 0].astype(np.float64), n, T, h, 0, 0)
    hh = h.astype(np.float64)[2 * n * (T - 1):]
    assert np.array_equal(g0, x[0, 0, :2 * n] * hh)


def test_out_of_range_delay_zeroes_the_spectrum():
    n, T, M = 32, 4, 24
    x, delays, phases, gains, h = _small_inputs(41, n, T, M, A=1)
    delays[0, 1, 5] = 40.6          # c = 41 > max_delay = 40
    delays[0, 0, 7] = -0.7          # c = -1
    delays[0, 0, 9] = np.nan
    r = _full_path(x, n, T, delays, phases, gains, h)
    assert r["invalid"] == 3
    assert r["valid"][0, 1, 5] == 0 and r["valid"][0, 0, 7] == 0 and r["valid"][0, 0, 9] == 0
    for p, F in ((1, 5), (0, 7), (0, 9)):
        assert not r["y"][0, p, F].any() and not r["q"][0, p, F].any()
    assert r["valid"].sum() == 2 * M - 3


# --------------------------------------------------------------------------
# Step 6 -- quantisation and corner turn (Sec. 2.1 item 6, Secs. 2.2, 3.6)
# --------------------------------------------------------------------------

def test_quantize_edge_table(golden_dir):
    vals, want = [], []
    for line in open(os.path.join(golden_dir, "quantize_edges.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v, q = line.split()
        vals.append(float(v))
        want.append(int(q))
    assert list(oracle.quantize(vals)) == want


def test_quantize_matches_rint_on_random_values():
    """numpy.rint rounds half to even: a textbook witness for the unsaturated range."""
    v = np.random.default_rng(4).uniform(-126.9, 126.9, 5000).astype(np.float32).astype(np.float64)
    v[:100] = np.arange(-50, 50) + 0.5       # exact ties
    assert np.array_equal(oracle.quantize(v), np.rint(v).astype(np.int8))


def test_heap_layout_round_trip():
    """out[a][F/S][k][F%S][p][c] = q[a][p][F][k][c], checked on distinct values."""
    A, M, n, S = 2, 8, 5, 4
    idx = np.arange(A * 2 * M * n * 2)
    q = (idx % 251 - 125).astype(np.int8).reshape(A, 2, M, n, 2)
    heap = oracle.heap_layout(q, S)
    for a in range(A):
        for p in range(2):
            for F in range(M):
                for k in range(n):
                    assert np.array_equal(heap[a, F // S, k, F % S, p], q[a, p, F, k])
    with pytest.raises(ValueError):
        oracle.heap_layout(q[:, :, :6], S)


def test_noise_output_level():
    """White noise of variance sigma^2 through taps with sum(h^2) = 1 gives
    spectra of per-component variance sigma^2/2 (Parseval through the PFB):
    the workload's sigma = 30 lands at about 21 LSB before the gain."""
    n, T = 256, 16
    w = synth.make_workload(synth.Shape(n=n, taps=T, antennas=1, samples=2 * n * 64), 8,
                            tone_channel=0)
    xn = np.random.default_rng(1).normal(0, 30, size=(1, 2, w.total))
    xn = np.clip(np.rint(xn), -511, 511).astype(np.int64)
    unit = np.zeros_like(w.gains)
    unit[..., 0] = 1
    r = _full_path(xn, n, T, np.zeros((1, 2, 64)), np.zeros((1, 2, 64)), unit, w.weights, 0)
    y = r["y"][:, :, T:, 1:]              # skip warm-up spectra and DC
    sd = np.sqrt(np.mean(y.real ** 2))
    assert 19.5 < sd < 22.5
