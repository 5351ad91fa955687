"""Streaming service (continuous batching over the C ABI).  Needs an MI355X.

* every feed's chunks, served mixed with other feeds' chunks under an HBM
  budget, come back bit-identical to the same chunks run alone through a
  plain stream (state carried on the device between chunks), whether they
  come from host memory or already sit in device memory;
* the served output matches the FP64 oracle on sampled spectra.
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

import paper_2303_09886_amd as fe            # noqa: E402
from paper_2303_09886_amd import service     # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def feeds_and_requests(n, T, S, feeds, chunks, kmax, seed):
    rng = np.random.default_rng(seed)
    unit = 2 * n * S
    plans, works, reqs = [], [], []
    for f in range(feeds):
        ks = rng.integers(1, kmax + 1, size=chunks)
        total = int(ks.sum()) * unit
        w = synth.make_workload(synth.Shape(n=n, taps=T, antennas=1, samples=total, spectra_per_heap=S),
                                500 + f)
        works.append(w)
        start = 0
        t = 0.0
        for k in ks:
            N = int(k) * unit
            raw, d, p = w.chunk(start, N)
            t += rng.exponential(2e-3)
            reqs.append(service.Request(f, raw[0], N, d[0], p[0], w.gains[0], arrival=t))
            plans.append((f, start, N))
            start += N
    return works, reqs


def alone(works, reqs, n, T, S, max_chunk, precision="fp32"):
    outs = {}
    reqs = [service.Request(r.feed, r.raw.cpu().numpy()[0] if torch.is_tensor(r.raw) else r.raw, r.n_samples,
                            r.delays.cpu().numpy()[0] if torch.is_tensor(r.delays) else r.delays,
                            r.phases.cpu().numpy()[0] if torch.is_tensor(r.phases) else r.phases,
                            r.gains.cpu().numpy()[0] if torch.is_tensor(r.gains) else r.gains)
            for r in reqs]
    for f, w in enumerate(works):
        st = fe.Stream(n, T, 1, w.weights, max_chunk, spectra_per_heap=S, precision=precision)
        for i, r in enumerate(reqs):
            if r.feed != f:
                continue
            M = r.n_samples // (2 * n)
            o = torch.empty((1, M // S, n, S, 2, 2), dtype=torch.int8, device="cuda")
            dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
            st.channelize(dv(r.raw[None]), r.n_samples, dv(r.delays[None]), dv(r.phases[None]),
                          dv(r.gains[None]), o)
            outs[i] = o.cpu().numpy()
        assert st.status() == fe.FE_OK
        st.close()
    return outs


@pytest.mark.parametrize("realtime,own_out", [(False, False), (True, False), (False, True),
                                               (False, "device"), (True, "device")])
def test_mixed_equals_alone(realtime, own_out):
    """own_out: the requests bring pinned output buffers (filled by the
    device directly instead of through the service's staging slots);
    "device": every buffer of the request, output included, is already in
    device memory (the device-resident service)."""
    n, T, S = 32768, 16, 16
    unit = 2 * n * S
    works, reqs = feeds_and_requests(n, T, S, feeds=3, chunks=4, kmax=3, seed=7)
    if own_out == "device":
        dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        for r in reqs:
            M = r.n_samples // (2 * n)
            r.raw, r.delays, r.phases, r.gains = dv(r.raw[None]), dv(r.delays[None]), dv(r.phases[None]), \
                dv(r.gains[None])
            r.out = torch.empty((1, M // S, n, S, 2, 2), dtype=torch.int8, device="cuda")
    elif own_out:
        for r in reqs:
            r.out = torch.empty(2 * r.n_samples, dtype=torch.int8).pin_memory()
    max_chunk = 3 * unit
    ref = alone(works, reqs, n, T, S, max_chunk)
    budget = 3 * service.chunk_device_bytes(n, max_chunk)        # about three chunks in flight
    svc = service.Service(n, T, works[0].weights, feeds=3, max_chunk_samples=max_chunk,
                          hbm_budget=budget, spectra_per_heap=S)
    stats = svc.run(reqs, realtime=realtime)
    svc.close()
    _say("  service (%s): %d chunks, %.2f Gsample/s, latency p50 %.2f ms p99 %.2f ms, peak %.0f MB in flight"
         % ("arrivals" if realtime else "backlog", stats["chunks"], stats["gsamples_per_s"],
            stats["latency_ms_p50"], stats["latency_ms_p99"], stats["peak_inflight_bytes"] / 1e6))
    for i, r in enumerate(reqs):
        if own_out == "device":
            got = r.out.cpu().numpy()
        else:
            got = r.out.numpy().reshape(ref[i].shape) if own_out else r.out
        assert got is not None and np.array_equal(got, ref[i]), i
    assert stats["peak_inflight_bytes"] <= budget


def test_fp16_feeds_mixed_equal_alone():
    """FP16 feeds (FP16 storage around the float32 two-level FFT at 32768
    channels), served mixed from device memory: bit-identical to the same
    chunks through plain FP16 streams."""
    n, T, S = 32768, 16, 16
    unit = 2 * n * S
    works, reqs = feeds_and_requests(n, T, S, feeds=2, chunks=3, kmax=3, seed=11)
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    for r in reqs:
        M = r.n_samples // (2 * n)
        r.raw, r.delays, r.phases, r.gains = dv(r.raw[None]), dv(r.delays[None]), dv(r.phases[None]), \
            dv(r.gains[None])
        r.out = torch.empty((1, M // S, n, S, 2, 2), dtype=torch.int8, device="cuda")
    max_chunk = 3 * unit
    ref = alone(works, reqs, n, T, S, max_chunk, precision="fp16")
    svc = service.Service(n, T, works[0].weights, feeds=2, max_chunk_samples=max_chunk,
                          hbm_budget=3 * service.chunk_device_bytes(n, max_chunk), spectra_per_heap=S,
                          precision="fp16")
    svc.run(reqs, realtime=False)
    svc.close()
    for i, r in enumerate(reqs):
        assert np.array_equal(r.out.cpu().numpy(), ref[i]), i


def test_served_output_matches_oracle():
    n, T, S = 32768, 16, 16
    unit = 2 * n * S
    works, reqs = feeds_and_requests(n, T, S, feeds=2, chunks=3, kmax=2, seed=9)
    svc = service.Service(n, T, works[0].weights, feeds=2, max_chunk_samples=2 * unit,
                          hbm_budget=1 << 40, spectra_per_heap=S)
    svc.run(reqs, realtime=False)
    svc.close()
    f = 0
    w = works[f]
    q = np.concatenate([r.out for r in reqs if r.feed == f], axis=1)      # [1][M/S][n][S][2][2]
    for F in (0, 15, 16, 40, q.shape[1] * S - 1):
        ref = oracle.channelize(w.raw, w.total, n, T, 128, w.weights, w.delays, w.phases, w.gains,
                                F, F + 1, want=("y", "q"))
        got = q[:, F // S, :, F % S]
        q_ref = ref["q"][:, :, 0].transpose(0, 2, 1, 3)
        v = ref["y"][:, :, 0].transpose(0, 2, 1)
        hard, _ = compare.int8_mismatches(got, q_ref, np.stack([v.real, v.imag], -1))
        assert hard == 0, F
