"""Batches of uneven streams (one graph launch per step) and the autotuner.
Needs an MI355X.

* a batch replayed from its HIP graph, step after step with new input in
  the captured buffers, gives bit for bit what each stream gives alone;
* so does the eager batch run (fork streams, no graph);
* every member's output from the replayed graph also matches the FP64
  oracle (the int8 bar of test_gpu_parity for FP32 members, 1 LSB for the
  matrix-core ones), with the launches grouped across members and without;
* autotuning changes launch shapes only: outputs are bit-identical, also
  for FIR runs longer than the FIR's per-workgroup delay table.
"""
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

SHAPES = [
    synth.Shape(n=1024, taps=8, antennas=1, samples=1 << 18, spectra_per_heap=16),
    synth.Shape(n=4096, taps=16, antennas=2, samples=1 << 19, spectra_per_heap=16),
    synth.Shape(n=8192, taps=24, antennas=1, samples=1 << 19, spectra_per_heap=16),
    synth.Shape(n=32768, taps=16, antennas=1, samples=1 << 20, spectra_per_heap=16),
    synth.Shape(n=1024, taps=16, antennas=1, samples=1 << 19, spectra_per_heap=16),
    synth.Shape(n=32768, taps=8, antennas=1, samples=1 << 20, spectra_per_heap=16),
]
PRECS = ["fp32", "fp32", "fp16", "fp32", "bf16", "fp16"]
STEPS = 2


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def make(shape, prec):
    return fe.Stream(shape.n, shape.taps, shape.antennas, workloads[shape][0].weights,
                     shape.samples, spectra_per_heap=shape.spectra_per_heap, precision=prec)


workloads = {s: (synth.make_workload(s, 40 + i, total=STEPS * s.samples),) for i, s in enumerate(SHAPES)}


def out_like(shape):
    M = shape.samples // (2 * shape.n)
    return torch.empty((shape.antennas, M // shape.spectra_per_heap, shape.n, shape.spectra_per_heap, 2, 2),
                       dtype=torch.int8, device="cuda")


def step_inputs(shape, step):
    w = workloads[shape][0]
    raw, d, p = w.chunk(step * shape.samples, shape.samples)
    return raw, d, p, w.gains


def alone():
    res = []
    for shape, prec in zip(SHAPES, PRECS):
        st = make(shape, prec)
        outs = []
        for k in range(STEPS):
            raw, d, p, g = step_inputs(shape, k)
            o = out_like(shape)
            st.channelize(dev(raw), shape.samples, dev(d), dev(p), dev(g), o)
            outs.append(o.cpu().numpy())
        assert st.status() == fe.FE_OK
        st.close()
        res.append(outs)
    return res


@pytest.mark.parametrize("grouped", [True, False])
def test_batch_graph_and_eager_match_streams_alone(grouped):
    ref = alone()
    for mode in ("graph", "eager"):
        members = [make(s, p) for s, p in zip(SHAPES, PRECS)]
        bufs = []
        for shape in SHAPES:
            raw, d, p, g = step_inputs(shape, 0)
            bufs.append([dev(raw), shape.samples, dev(d), dev(p), dev(g), out_like(shape)])
        batch = fe.Batch(members)
        batch.set_grouped(grouped)
        if mode == "graph":
            batch.capture(bufs)
        for k in range(STEPS):
            for shape, b in zip(SHAPES, bufs):
                raw, d, p, _ = step_inputs(shape, k)
                b[0].copy_(torch.from_numpy(raw))
                b[2].copy_(torch.from_numpy(d))
                b[3].copy_(torch.from_numpy(p))
            torch.cuda.synchronize()
            if mode == "graph":
                batch.launch()
            else:
                batch.run(bufs)
            torch.cuda.synchronize()
            for i, b in enumerate(bufs):
                assert np.array_equal(b[5].cpu().numpy(), ref[i][k]), (mode, i, k)
        batch.close()
        for m in members:
            assert m.status() == fe.FE_OK
            m.close()
        _say("  batch %s (grouped %s): %d uneven streams x %d steps bit-identical to the streams alone"
             % (mode, grouped, len(SHAPES), STEPS))


@pytest.mark.parametrize("grouped", [True, False])
def test_every_batch_member_matches_oracle(grouped):
    """Each member's output from the graph-replayed batch (grouped launches
    and per-member fork streams), over both steps, against the FP64 oracle:
    the int8 rule of
    test_gpu_parity for FP32 members, within 1 LSB for the FP16/BF16
    members (the matrix-core bar of test_gpu_mfma)."""
    members = [make(s, p) for s, p in zip(SHAPES, PRECS)]
    bufs = []
    for shape in SHAPES:
        raw, d, p, g = step_inputs(shape, 0)
        bufs.append([dev(raw), shape.samples, dev(d), dev(p), dev(g), out_like(shape)])
    batch = fe.Batch(members)
    batch.set_grouped(grouped)
    batch.capture(bufs)
    outs = [[] for _ in SHAPES]
    for k in range(STEPS):
        for shape, b in zip(SHAPES, bufs):
            raw, d, p, _ = step_inputs(shape, k)
            b[0].copy_(torch.from_numpy(raw))
            b[2].copy_(torch.from_numpy(d))
            b[3].copy_(torch.from_numpy(p))
        torch.cuda.synchronize()
        batch.launch()
        torch.cuda.synchronize()
        for i, b in enumerate(bufs):
            outs[i].append(b[5].cpu().numpy())
    batch.close()
    for m in members:
        assert m.status() == fe.FE_OK
        m.close()
    for i, (shape, prec) in enumerate(zip(SHAPES, PRECS)):
        w = workloads[shape][0]
        S = shape.spectra_per_heap
        r = oracle.channelize(w.raw, w.total, shape.n, shape.taps, 128, w.weights, w.delays, w.phases,
                              w.gains, want=("y", "q"))
        q = np.concatenate(outs[i], axis=1)
        q_ref = oracle.heap_layout(r["q"], S)
        if prec == "fp32":
            hard, soft = compare.int8_mismatches(q, q_ref, compare.heap_values(r["y"], S))
            _say("  member %d (n=%d T=%d %s): %d hard, %d boundary differences"
                 % (i, shape.n, shape.taps, prec, hard, soft))
            assert hard == 0
        else:
            dq = np.abs(q.astype(np.int16) - q_ref.astype(np.int16))
            _say("  member %d (n=%d T=%d %s): max |dq| %d" % (i, shape.n, shape.taps, prec, dq.max()))
            assert dq.max() <= 1


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_autotune_keeps_results(prec):
    # FP16: 1024 spectra, 4 tiles of the matrix-core FIR, so chains of 1, 2 and 4 tiles differ
    shape = synth.Shape(n=4096, taps=16, antennas=2, samples=1 << (21 if prec == "fp32" else 23),
                        spectra_per_heap=16)
    w = synth.make_workload(shape, 8)
    raw, d, p = w.chunk(0, shape.samples)
    args = [dev(raw), shape.samples, dev(d), dev(p), dev(w.gains)]
    outs = []
    for tune in (False, True):
        st = fe.Stream(shape.n, shape.taps, shape.antennas, w.weights, shape.samples, spectra_per_heap=16,
                       precision=prec)
        o = out_like(shape)
        if tune:
            choice = st.autotune(*args, o, iters=2)
            _say("  autotune chose FIR run length %d" % choice)
        st.channelize(*args, o)
        outs.append(o.cpu().numpy())
        assert st.status() == fe.FE_OK
        st.close()
    assert np.array_equal(outs[0], outs[1])
    for fb in (1, 2, 8):
        st = fe.Stream(shape.n, shape.taps, shape.antennas, w.weights, shape.samples, spectra_per_heap=16,
                       precision=prec)
        st.set_tuning(fb)
        o = out_like(shape)
        st.channelize(*args, o)
        assert np.array_equal(o.cpu().numpy(), outs[0])
        st.close()


def test_two_level_split_keeps_results():
    """The two-level FFT's post kernel with a spectrum's rounds over 1, 3
    or 9 workgroups, and as autotuned: bit-identical int8 output (16384
    channels, 64 spectra per call: 128 spectrum-polarizations)."""
    shape = synth.Shape(n=16384, taps=16, antennas=1, samples=2 * 16384 * 64, spectra_per_heap=16)
    w = synth.make_workload(shape, 12)
    raw, d, p = w.chunk(0, shape.samples)
    args = [dev(raw), shape.samples, dev(d), dev(p), dev(w.gains)]
    outs = []
    for parts in (0, 1, 3, 9, "tuned"):
        st = fe.Stream(shape.n, shape.taps, 1, w.weights, shape.samples, spectra_per_heap=16)
        o = out_like(shape)
        if parts == "tuned":
            st.autotune(*args, o, iters=2)
            _say("  autotune chose %d workgroups per spectrum (0 = per call)" % st.fft_parts())
        else:
            st.set_fft_parts(parts)
            assert st.fft_parts() == parts
        st.channelize(*args, o)
        assert st.status() == fe.FE_OK
        outs.append(o.cpu().numpy())
        st.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_fir_runs_longer_than_the_delay_table():
    """FIR run lengths of 64 .. 4096 spectra over 2048 spectra whose coarse
    delay steps every ~100 spectra: runs cross the 1024-spectrum segments of
    the FIR's delay table, some with a delay that continues across the seam.
    Each output is formed by the same arithmetic whatever the run length, so
    the results are bit-identical, and they match the oracle."""
    shape = synth.Shape(n=256, taps=16, antennas=1, samples=1 << 20, spectra_per_heap=16)
    w = synth.make_workload(shape, 9, delay_rate=1e-4)
    raw, d, p = w.chunk(0, shape.samples)
    args = [dev(raw), shape.samples, dev(d), dev(p), dev(w.gains)]
    outs = []
    for fb in (0, 1, 16, 64):
        _say("  FIR run length %d batches" % fb)
        st = fe.Stream(shape.n, shape.taps, shape.antennas, w.weights, shape.samples, spectra_per_heap=16)
        st.set_tuning(fb)
        o = out_like(shape)
        st.channelize(*args, o)
        assert st.status() == fe.FE_OK
        outs.append(o.cpu().numpy())
        st.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    r = oracle.channelize(w.raw, w.total, shape.n, shape.taps, 128, w.weights, w.delays, w.phases,
                          w.gains, want=("y", "q"))
    hard, soft = compare.int8_mismatches(outs[0], oracle.heap_layout(r["q"], 16),
                                         compare.heap_values(r["y"], 16))
    assert hard == 0
