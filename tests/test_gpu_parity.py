"""Parity of the HIP channelizer with the FP64 oracle (needs an MI355X).

All calls go through the C ABI (ctypes binding).  Inputs are seeded and
synthetic (synth).  Tolerances (oracle.compare): unpack and coarse delay
bit-exact; pre-quantisation spectra within 1e-5 relative; int8 exact except
within 1e-3 of a rounding boundary, where +-1 is allowed.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import compare

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2303_09886_amd as fe   # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# Every stream test runs on each kernel path (fe_stream_set_schedule): the
# split path (FIR kernel, filtered samples in device memory, FFT/post kernel,
# corner turn), the fused kernel (FP32, n <= 4096, T <= 16) and the split
# path whose FFT/post kernel writes the heaps itself (FP32, n <= 8192);
# shapes a path cannot run run split either way.
PATH = {"now": "split"}


@pytest.fixture(autouse=True, params=["split", "fused", "split_folded"])
def kernel_path(request):
    PATH["now"] = request.param
    _say("[path %s]" % request.param)
    yield request.param
    PATH["now"] = "split"


def make_stream(w, max_samples, max_delay=128):
    s = w.shape
    return fe.Stream(s.n, s.taps, s.antennas, w.weights, max_samples,
                     spectra_per_heap=s.spectra_per_heap, max_delay=max_delay, path=PATH["now"])


def gpu_run(w, chunk, mode="int8", max_delay=128, stream=None):
    """Feed the workload to a fresh stream in calls of ``chunk`` samples;
    return the concatenated output of the requested kind."""
    s = w.shape
    A, n, S = s.antennas, s.n, s.spectra_per_heap
    st = stream or make_stream(w, chunk, max_delay)
    gains = dev(w.gains)
    outs = []
    for start in range(0, w.total, chunk):
        raw, d, p = w.chunk(start, chunk)
        M = chunk // (2 * n)
        raw_t, d_t, p_t = dev(raw), dev(d), dev(p)
        if mode == "int8":
            o = torch.empty((A, M // S, n, S, 2, 2), dtype=torch.int8, device="cuda")
            st.channelize(raw_t, chunk, d_t, p_t, gains, o)
        elif mode == "prequant":
            o = torch.empty((A, 2, M, n, 2), dtype=torch.float32, device="cuda")
            st.channelize_prequant(raw_t, chunk, d_t, p_t, gains, o)
        else:
            o = torch.empty((A, 2, M, 2 * n), dtype=torch.float32, device="cuda")
            st.channelize_fir(raw_t, chunk, d_t, o)
        torch.cuda.synchronize()
        outs.append(o.cpu().numpy())
    status = st.status()
    if stream is None:
        st.close()
    axis = 1 if mode == "int8" else 2
    out = np.concatenate(outs, axis=axis)
    if mode == "prequant":
        out = out[..., 0] + 1j * out[..., 1]
    return out, status


def oracle_run(w, want=("y", "q"), max_delay=128):
    s = w.shape
    return oracle.channelize(w.raw, w.total, s.n, s.taps, max_delay, w.weights, w.delays,
                             w.phases, w.gains, want=want)


def check_int8(q_gpu, ref, S, context=""):
    q_ref = oracle.heap_layout(ref["q"], S)
    v_ref = compare.heap_values(ref["y"], S)
    hard, soft = compare.int8_mismatches(q_gpu, q_ref, v_ref)
    _say("int8 %s: %d hard mismatches, %d boundary differences of %d values"
         % (context, hard, soft, q_ref.size))
    assert hard == 0
    return soft


# --------------------------------------------------------------------------
# Step 1 alone: the device unpacker is bit-exact
# --------------------------------------------------------------------------

def test_unpack_bit_exact():
    rng = np.random.default_rng(7)
    raw = rng.integers(0, 256, size=(1 << 17) * 5, dtype=np.uint8)
    count = raw.size * 8 // 10
    out = torch.empty(count, dtype=torch.int32, device="cuda")
    fe.debug_unpack10(dev(raw), 0, count, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle.unpack10(raw, 0, count))
    for first in (1, 2, 3, 5, 1001):
        o = torch.empty(777, dtype=torch.int32, device="cuda")
        fe.debug_unpack10(dev(raw), first, 777, o)
        torch.cuda.synchronize()
        assert np.array_equal(o.cpu().numpy(), oracle.unpack10(raw, first, 777))
    codes = np.arange(-512, 512)
    for lead in range(4):
        x = np.concatenate([np.zeros(lead, dtype=np.int64), codes, np.zeros(4 - lead, dtype=np.int64)])
        packed = synth.pack10(x)
        o = torch.empty(x.size, dtype=torch.int32, device="cuda")
        fe.debug_unpack10(dev(packed), 0, x.size, o)
        torch.cuda.synchronize()
        assert np.array_equal(o.cpu().numpy(), x)


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_hot_path_unpack_every_code_and_phase(prec):
    """The unpackers inside the FIR kernels, bit for bit: with one tap of
    value 1 the filtered sample is the sample itself, g_{F,t} = s_{2nF+t-c_F}
    (Eq. (1) with T = 1), exactly in every precision (10-bit codes are exact
    in FP16 and in BF16 hi+lo).  The stream repeats the 1024 codes with
    period 1025, so every code sits at every bit phase (10 i mod 8); the
    integer delays step through 0 .. 120 and three calls put the history seam
    under the first spectra of the later calls."""
    _say("hot-path unpack %s" % prec)
    n, S, M, calls = 256, 4, 32, 3
    shape = synth.Shape(n=n, taps=1, antennas=2, samples=2 * n * M, spectra_per_heap=S)
    w = synth.make_workload(shape, 11, total=2 * n * M * calls)
    i = np.arange(w.total)
    x = np.empty_like(w.x)
    for a in range(2):
        for p in range(2):
            x[a, p] = (i + 257 * (2 * a + p)) % 1025 % 1024 - 512
    w.x, w.raw = x, synth.pack10(x)
    w.weights = np.ones_like(w.weights)
    F = np.arange(M * calls)
    w.delays[:] = ((F * 7 + 13 * np.arange(4).reshape(2, 2, 1)) % 121).astype(np.float64)
    # FP32 streams on the split and the fused kernels; FP16/BF16 streams on
    # the vector FIR (under "split") and the matrix-core FIR (under "fused")
    path = PATH["now"] if prec == "fp32" else {"fused": "matrix_fir"}.get(PATH["now"], "split")
    st = fe.Stream(n, 1, 2, w.weights, 2 * n * M, spectra_per_heap=S, precision=prec, path=path)
    g, status = gpu_run(w, 2 * n * M, mode="fir", stream=st)
    st.close()
    assert status == fe.FE_OK
    ref = oracle_run(w, want=("g",))
    assert np.array_equal(g, ref["g"].astype(np.float32))
    # the window of spectrum F really is the stream shifted by c_F
    assert np.array_equal(ref["g"][1, 0, 40], x[1, 0, 2 * n * 40 - int(w.delays[1, 0, 40]) + np.arange(2 * n)])


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_hot_path_unpack_at_zero_delay(prec):
    """With coarse delay 0 the last column pair of a region's last row ends at
    its last byte, where the FIR reads that pair's word a byte early and
    shifts it back (a whole-word load would pass the end): every code at every
    bit phase again, all delays 0, over the call's own rows and the history
    seam."""
    _say("hot-path unpack at zero delay %s" % prec)
    n, S, M, calls = 256, 4, 32, 3
    shape = synth.Shape(n=n, taps=1, antennas=2, samples=2 * n * M, spectra_per_heap=S)
    w = synth.make_workload(shape, 12, total=2 * n * M * calls)
    i = np.arange(w.total)
    x = np.empty_like(w.x)
    for a in range(2):
        for p in range(2):
            x[a, p] = (i + 311 * (2 * a + p)) % 1025 % 1024 - 512
    w.x, w.raw = x, synth.pack10(x)
    w.weights = np.ones_like(w.weights)
    w.delays[:] = 0.0
    path = PATH["now"] if prec == "fp32" else {"fused": "matrix_fir"}.get(PATH["now"], "split")
    st = fe.Stream(n, 1, 2, w.weights, 2 * n * M, spectra_per_heap=S, precision=prec, path=path)
    g, status = gpu_run(w, 2 * n * M, mode="fir", stream=st)
    st.close()
    assert status == fe.FE_OK
    ref = oracle_run(w, want=("g",))
    assert np.array_equal(g, ref["g"].astype(np.float32))


# --------------------------------------------------------------------------
# Steps 1-3a: FIR output with impulses is exact; with noise within 1e-5
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,T,step", [(1024, 16, 5), (256, 4, 5), (4096, 16, 5), (512, 24, 5),
                                      (2048, 3, 5), (1024, 16, 0), (256, 32, 0), (512, 8, 40),
                                      (256, 16, 16), (1024, 8, 8), (512, 16, 48)])
def test_fir_impulses_bit_exact(n, T, step):
    """One impulse per window: g must equal float32(value * h[u]) exactly,
    which pins the sample order, the coarse-delay index and the tap mapping.
    step = spectra between integer-delay steps (0: constant delay)."""
    _say("fir impulses n=%d T=%d step=%d" % (n, T, step))
    S, A = 4, 2
    M = 32 * S if step != 5 else 8 * S
    shape = synth.Shape(n=n, taps=T, antennas=A, samples=2 * n * M, spectra_per_heap=S)
    w = synth.make_workload(shape, 99)
    x = np.zeros_like(w.x)
    rng = np.random.default_rng(n + T)
    spacing = 2 * n * (T + 2)
    for a in range(A):
        for p in range(2):
            pos = np.arange(rng.integers(0, 2 * n), w.total, spacing)
            x[a, p, pos] = rng.choice([-512, 511, 1, -1, 300], size=pos.size)
    w.x, w.raw = x, synth.pack10(x)
    ramp = np.floor(np.arange(M) / step) if step else np.zeros(M)
    w.delays[:] = np.floor(rng.uniform(0, 100, size=(A, 2, 1))) + ramp[None, None, :]
    g, status = gpu_run(w, w.total, mode="fir")
    assert status == fe.FE_OK
    ref = oracle_run(w, want=("g",))
    assert np.array_equal(g, ref["g"].astype(np.float32))


@pytest.mark.parametrize("n,T,step", [(1024, 16, 1), (512, 16, 2), (256, 24, 3), (256, 32, 2),
                                      (1024, 16, 4), (512, 8, 1)])
def test_fir_short_spans_bit_exact(n, T, step):
    """Integer-delay steps every 1-4 spectra: spans of one delay shorter
    than a group take the one-output-at-a-time path; impulses pin it
    exactly as in test_fir_impulses_bit_exact."""
    _say("fir short spans n=%d T=%d step=%d" % (n, T, step))
    S, A, M = 4, 2, 40
    shape = synth.Shape(n=n, taps=T, antennas=A, samples=2 * n * M, spectra_per_heap=S)
    w = synth.make_workload(shape, 77)
    x = np.zeros_like(w.x)
    rng = np.random.default_rng(n + 3 * T + step)
    spacing = 2 * n * (T + 2) + 3
    for a in range(A):
        for p in range(2):
            pos = np.arange(rng.integers(0, 2 * n), w.total, spacing)
            x[a, p, pos] = rng.choice([-512, 511, 1, -1, 300], size=pos.size)
    w.x, w.raw = x, synth.pack10(x)
    ramp = np.floor(np.arange(M) / step)
    w.delays[:] = np.floor(rng.uniform(0, 60, size=(A, 2, 1))) + ramp[None, None, :]
    g, status = gpu_run(w, w.total, mode="fir")
    assert status == fe.FE_OK
    ref = oracle_run(w, want=("g",))
    assert np.array_equal(g, ref["g"].astype(np.float32))


@pytest.mark.parametrize("n,T,A,S,M", [(1024, 16, 1, 4, 44), (4096, 16, 2, 4, 36), (256, 8, 3, 2, 70)])
def test_fir_matches_oracle(n, T, A, S, M):
    _say("fir noise n=%d T=%d A=%d M=%d" % (n, T, A, M))
    shape = synth.Shape(n=n, taps=T, antennas=A, samples=2 * n * M, spectra_per_heap=S)
    w = synth.make_workload(shape, 5)
    g, _ = gpu_run(w, w.total, mode="fir")
    ref = oracle_run(w, want=("g",))
    nw, el = compare.prequant_errors(g, ref["g"])
    _say("  g normwise %.3g elementwise %.3g" % (nw, el))
    assert nw <= 1e-5 and el <= 1e-5


# --------------------------------------------------------------------------
# Whole path against the oracle
# --------------------------------------------------------------------------

CASES = [
    # n, T, A, S_h, M (spectra per call), calls
    (1024, 16, 1, 4, 44, 1),
    (4096, 16, 2, 4, 36, 1),
    (256, 4, 3, 8, 64, 2),
    (512, 24, 1, 2, 30, 2),
    (2048, 32, 1, 4, 40, 1),
    (8192, 8, 1, 2, 18, 1),
    (1024, 13, 2, 8, 48, 3),
    (1024, 1, 1, 4, 20, 1),
    # long runs of constant delay: the FIR's grouped fast path, T = 4 .. 32
    (256, 4, 1, 32, 256, 1),
    (256, 8, 2, 32, 192, 2),
    (512, 16, 1, 64, 256, 1),
    (256, 24, 1, 32, 256, 1),
    (256, 32, 1, 64, 256, 1),
    # channel counts above one workgroup's LDS: two-level FFT; calls shorter
    # than the history
    (16384, 16, 1, 2, 10, 2),
    (32768, 8, 2, 2, 6, 1),
    (32768, 16, 1, 2, 4, 3),
    # two-level FFT behind each FIR form: more than 16 taps (the first
    # radix-16 stage in a pass of its own), and 4 and 13 taps (the FIR does
    # that stage itself)
    (16384, 24, 1, 2, 8, 2),
    (16384, 32, 2, 2, 6, 1),
    (16384, 4, 1, 4, 16, 1),
    (32768, 13, 1, 2, 6, 2),
]


@pytest.mark.parametrize("n,T,A,S,M,calls", CASES)
def test_prequant_matches_oracle(n, T, A, S, M, calls):
    _say("prequant n=%d T=%d A=%d S=%d M=%d calls=%d" % (n, T, A, S, M, calls))
    shape = synth.Shape(n=n, taps=T, antennas=A, samples=2 * n * M, spectra_per_heap=S)
    w = synth.make_workload(shape, 1000 + n + T, total=2 * n * M * calls)
    y, status = gpu_run(w, 2 * n * M, mode="prequant")
    assert status == fe.FE_OK
    ref = oracle_run(w, want=("y",))
    if n <= 8192:
        nw, el = compare.assert_prequant_close(y, ref["y"])
    else:
        # 65536-point transforms: the normwise bar stays 1e-5; the
        # elementwise bar is 3e-5.  FP32 rounding alone reaches ~6.5e-6
        # elementwise here (a single-precision library rfft of the oracle's
        # own filtered samples, same data), before the FIR and the
        # rotation/gain add theirs
        nw, el = compare.prequant_errors(y, ref["y"])
        assert nw <= compare.PREQUANT_RTOL
        assert el <= 3 * compare.PREQUANT_RTOL
    _say("  Y normwise %.3g elementwise %.3g" % (nw, el))


# odd heap sizes: heaps of 3 and 1 spectra (the FFT/post kernel then writes
# one spectrum's bytes per channel at a time)
ODD_HEAPS = [(1024, 16, 2, 3, 33, 2), (8192, 8, 1, 1, 7, 1)]
# the two-level FFT's rounds split over 3 workgroups (128 spectra-pols) and
# kept in one (512)
TWO_LEVEL_SPLITS = [(16384, 8, 1, 4, 64, 1), (16384, 16, 2, 2, 128, 1)]


@pytest.mark.parametrize("n,T,A,S,M,calls", CASES[:4] + CASES[8:10] + CASES[13:15] + CASES[16:]
                         + ODD_HEAPS + TWO_LEVEL_SPLITS)
def test_int8_matches_oracle(n, T, A, S, M, calls):
    _say("int8 n=%d T=%d A=%d S=%d M=%d calls=%d" % (n, T, A, S, M, calls))
    shape = synth.Shape(n=n, taps=T, antennas=A, samples=2 * n * M, spectra_per_heap=S)
    w = synth.make_workload(shape, 2000 + n + T, total=2 * n * M * calls)
    q, status = gpu_run(w, 2 * n * M, mode="int8")
    assert status == fe.FE_OK
    ref = oracle_run(w)
    check_int8(q, ref, S, "n=%d" % n)


def test_calls_shorter_than_history():
    """N < H: the history is shifted rather than replaced."""
    n, T, S = 256, 16, 2
    shape = synth.Shape(n=n, taps=T, antennas=2, samples=2 * n * S, spectra_per_heap=S)
    w = synth.make_workload(shape, 77, total=2 * n * S * 20)
    q, status = gpu_run(w, 2 * n * S, mode="int8")
    assert status == fe.FE_OK
    ref = oracle_run(w)
    check_int8(q, ref, S, "short calls")
    y, _ = gpu_run(w, 2 * n * S, mode="prequant")
    compare.assert_prequant_close(y, ref["y"])


def test_chunking_is_invisible_and_deterministic():
    """One call of 4N equals four calls of N bit for bit; reruns are identical."""
    n, T, S = 1024, 16, 4
    shape = synth.Shape(n=n, taps=T, antennas=2, samples=2 * n * S * 4, spectra_per_heap=S)
    w = synth.make_workload(shape, 3)
    q1, _ = gpu_run(w, w.total)
    q4, _ = gpu_run(w, w.total // 4)
    q1b, _ = gpu_run(w, w.total)
    assert np.array_equal(q1, q4)
    assert np.array_equal(q1, q1b)


@pytest.mark.parametrize("n", [1024, 16384])
def test_out_of_range_delay_sets_status_and_zeroes(n):
    """Invalid delays zero their spectra and raise the sticky status; at
    16384 channels the FIR that also does the first FFT stage takes its
    per-spectrum path for them."""
    T, S, M = 16, 4, 16
    shape = synth.Shape(n=n, taps=T, antennas=1, samples=2 * n * M, spectra_per_heap=S)
    w = synth.make_workload(shape, 4)
    w.delays[0, 1, 5] = 128.7          # c = 129 > max_delay
    w.delays[0, 0, 9] = np.nan
    w.delays[0, 0, 11] = -3.0
    y, status = gpu_run(w, w.total, mode="prequant")
    assert status == fe.FE_EDELAY
    ref = oracle_run(w, want=("y", "valid"))
    assert ref["invalid"] == 3
    assert not y[0, 1, 5].any() and not y[0, 0, 9].any() and not y[0, 0, 11].any()
    compare.assert_prequant_close(y, ref["y"])
    # reset clears the sticky status
    st = make_stream(w, w.total)
    raw, d, p = w.chunk(0, w.total)
    o = torch.empty((1, 2, M, n, 2), dtype=torch.float32, device="cuda")
    st.channelize_prequant(dev(raw), w.total, dev(d), dev(p), dev(w.gains), o)
    assert st.status() == fe.FE_EDELAY
    st.reset()
    assert st.status() == fe.FE_OK
    st.close()


def test_host_validation_with_live_stream():
    n, T, S, M = 1024, 16, 4, 8
    shape = synth.Shape(n=n, taps=T, antennas=1, samples=2 * n * M, spectra_per_heap=S)
    w = synth.make_workload(shape, 4)
    st = make_stream(w, w.total)
    raw, d, p = w.chunk(0, w.total)
    o = torch.empty((1, M // S, n, S, 2, 2), dtype=torch.int8, device="cuda")
    with pytest.raises(fe.FEngineError) as e:
        st.channelize(dev(raw), w.total // 2 + 2 * n, dev(d), dev(p), dev(w.gains), o)
    assert e.value.status == fe.FE_EINVAL
    # more samples than the stream was created for: the library refuses the
    # call (the buffers are large enough, so the binding passes it on)
    raw2 = np.concatenate([raw, raw], axis=-1)
    d2, p2 = np.concatenate([d, d], axis=-1), np.concatenate([p, p], axis=-1)
    o2 = torch.empty((1, 2 * M // S, n, S, 2, 2), dtype=torch.int8, device="cuda")
    with pytest.raises(fe.FEngineError) as e:
        st.channelize(dev(raw2), 2 * w.total, dev(d2), dev(p2), dev(w.gains), o2)
    assert e.value.status == fe.FE_ESIZE
    # an empty call is not a whole number of heaps either
    with pytest.raises(fe.FEngineError) as e:
        st.channelize(dev(raw), 0, dev(d), dev(p), dev(w.gains), o)
    assert e.value.status == fe.FE_EINVAL
    assert st.status() == fe.FE_OK                 # refused calls leave the stream untouched
    st.close()


@pytest.mark.parametrize("T", [16, 32])
def test_largest_delay_matches_oracle(T):
    """Coarse delays at the largest allowed value D (d in [D - 0.5, D + 0.5))
    and just below it, over two calls: the FIR reads the most history rows
    and the stream keeps the deepest tail."""
    n, S, M, calls, D = 256, 4, 48, 2, 128
    _say("largest delay T=%d" % T)
    shape = synth.Shape(n=n, taps=T, antennas=1, samples=2 * n * M, spectra_per_heap=S)
    w = synth.make_workload(shape, 31 + T, total=2 * n * M * calls)
    F = np.arange(w.delays.shape[2])
    w.delays[0, 0] = D + 0.49 - 0.98 * (F % 7) / 7.0      # c = D throughout
    w.delays[0, 1] = D - 0.51 + 0.3 * (F % 2)              # c alternates D - 1, D
    y, status = gpu_run(w, 2 * n * M, mode="prequant", max_delay=D)
    assert status == fe.FE_OK
    ref = oracle_run(w, want=("y", "q"), max_delay=D)
    nw, el = compare.assert_prequant_close(y, ref["y"])
    _say("  Y normwise %.3g elementwise %.3g" % (nw, el))
    q, status = gpu_run(w, 2 * n * M, mode="int8", max_delay=D)
    assert status == fe.FE_OK
    check_int8(q, ref, S, "largest delay")


# --------------------------------------------------------------------------
# Full-size configurations, in the launch configuration the benchmark times
# --------------------------------------------------------------------------

def test_small_config_full():
    """1 antenna x 2 pols, 2^20 samples/pol, 1024 channels, 16 taps: every output."""
    _say("small config, full comparison")
    w = synth.make_workload(synth.SMALL, 1)
    q, status = gpu_run(w, w.total, mode="int8")
    assert status == fe.FE_OK
    ref = oracle_run(w)
    check_int8(q, ref, synth.SMALL.spectra_per_heap, "small config")
    y, _ = gpu_run(w, w.total, mode="prequant")
    nw, el = compare.assert_prequant_close(y, ref["y"])
    _say("  Y normwise %.3g elementwise %.3g" % (nw, el))


def test_large_config_every_spectrum():
    """4 antennas x 2 pols, 2^24 samples/pol, 4096 channels, 16 taps (the
    benchmark's workload): every spectrum of the int8 heaps against the
    int8 rule and every pre-quantisation spectrum within the 1e-5 bars.  The
    oracle runs per antenna and heap on a thread pool (its ctypes calls
    release the interpreter lock)."""
    import concurrent.futures as cf
    _say("large config, every spectrum")
    w = synth.make_workload(synth.LARGE, 2)
    shape = w.shape
    q, status = gpu_run(w, w.total, mode="int8")
    assert status == fe.FE_OK
    y, status = gpu_run(w, w.total, mode="prequant")
    assert status == fe.FE_OK
    S, n, A = shape.spectra_per_heap, shape.n, shape.antennas
    M = w.total // (2 * n)

    def check(task):
        a, h = task
        F0, F1 = h * S, (h + 1) * S
        ref = oracle.channelize(w.raw[a:a + 1], w.total, n, shape.taps, 128, w.weights, w.delays[a:a + 1],
                                w.phases[a:a + 1], w.gains[a:a + 1], F0, F1, want=("y", "q"))
        hard, soft = compare.int8_mismatches(q[a:a + 1, h:h + 1], oracle.heap_layout(ref["q"], S),
                                             compare.heap_values(ref["y"], S))
        nw, el = compare.prequant_errors(y[a:a + 1, :, F0:F1], ref["y"])
        return a, h, hard, soft, nw, el

    tasks = [(a, h) for a in range(A) for h in range(M // S)]
    with cf.ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1))) as ex:
        res = list(ex.map(check, tasks))
    hard = sum(r[2] for r in res)
    soft = sum(r[3] for r in res)
    nw = max(r[4] for r in res)
    el = max(r[5] for r in res)
    _say("  %d heaps: %d hard, %d boundary int8 differences; Y normwise %.3g elementwise %.3g"
         % (len(res), hard, soft, nw, el))
    assert hard == 0
    assert nw <= compare.PREQUANT_RTOL and el <= compare.PREQUANT_RTOL
