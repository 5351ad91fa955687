"""fe_channelize_noalloc (static device scratch, no allocation) against
fe_channelize on the same inputs: two calls in a row, the second smaller,
through the C ABI.  Same kernels, same arithmetic: the outputs and the
stream state must be identical, bit for bit.  Needs an MI355X."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2303_09886_amd as fe   # noqa: E402
from paper_2303_09886_amd.fengine import FE_NOALLOC_SCRATCH_BYTES   # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run(st, w, calls, noalloc):
    """Consecutive calls of calls[i] samples; int8 heaps of each call."""
    s = w.shape
    A, n, S = s.antennas, s.n, s.spectra_per_heap
    gains = dev(w.gains)
    outs, start = [], 0
    for N in calls:
        raw, d, p = w.chunk(start, N)
        M = N // (2 * n)
        o = torch.full((A, M // S, n, S, 2, 2), 77, dtype=torch.int8, device="cuda")
        f = st.channelize_noalloc if noalloc else st.channelize
        f(dev(raw), N, dev(d), dev(p), gains, o)
        torch.cuda.synchronize()
        outs.append(o.cpu().numpy())
        start += N
    return outs, st.status()


# (n, T, antennas, precision, path, samples of call 1, samples of call 2):
# the split, folded and fused FP32 paths, the matrix-core paths (turn
# separate and folded), the two-level FFT, and second calls shorter than the
# history (its assembly buffer)
CASES = [
    (1024, 16, 2, "fp32", "split", 2 * 1024 * 64, 2 * 1024 * 16),
    (2048, 16, 2, "fp32", "split_folded", 2 * 2048 * 32, 2 * 2048 * 8),
    (1024, 8, 1, "fp32", "fused", 2 * 1024 * 64, 2 * 1024 * 8),
    (512, 16, 1, "fp16", "auto", 2 * 512 * 96, 2 * 512 * 32),
    (1024, 16, 1, "bf16", "split_folded", 2 * 1024 * 64, 2 * 1024 * 16),
    (16384, 16, 1, "fp32", "auto", 2 * 16384 * 32, 2 * 16384 * 16),
    (256, 16, 1, "fp32", "split", 2 * 256 * 64, 2 * 256 * 4),
]


@pytest.mark.parametrize("n,T,A,prec,path,N1,N2", CASES)
def test_noalloc_matches_channelize(n, T, A, prec, path, N1, N2):
    _say("noalloc n=%d T=%d A=%d %s %s calls %d, %d" % (n, T, A, prec, path, N1, N2))
    S = 4 if n <= 4096 else 16
    shape = synth.Shape(n=n, taps=T, antennas=A, samples=N1, spectra_per_heap=S)
    w = synth.make_workload(shape, 501 + n + T, total=N1 + N2)
    outs = []
    for noalloc in (False, True):
        st = fe.Stream(n, T, A, w.weights, N1, spectra_per_heap=S, precision=prec, path=path)
        outs.append(run(st, w, [N1, N2], noalloc))
        st.close()
    (ref, st_ref), (got, st_got) = outs
    assert st_ref == st_got == fe.FE_OK
    for i, (a, b) in enumerate(zip(ref, got)):
        assert a.shape == b.shape
        assert np.array_equal(a, b), "call %d differs in %d values" % (i, int((a != b).sum()))


def test_noalloc_refuses_calls_beyond_the_scratch():
    # 4 antennas x 2 pols x 2^21 samples need 5 x 2^24 bytes (g + int8) > 64 MiB
    n, T, A, N = 1024, 16, 4, 1 << 21
    need = 2 * A * N * 5
    assert need > FE_NOALLOC_SCRATCH_BYTES
    shape = synth.Shape(n=n, taps=T, antennas=A, samples=N)
    w = synth.make_workload(shape, 9)
    st = fe.Stream(n, T, A, w.weights, N, path="split")
    M = N // (2 * n)
    o = torch.empty((A, M // 256, n, 256, 2, 2), dtype=torch.int8, device="cuda")
    with pytest.raises(fe.FEngineError) as e:
        st.channelize_noalloc(dev(w.raw), N, dev(w.delays), dev(w.phases), dev(w.gains), o)
    assert e.value.status == fe.FE_ESIZE
    assert st.status() == fe.FE_OK          # nothing was enqueued
    st.close()
