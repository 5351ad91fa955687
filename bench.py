#!/usr/bin/env python3
"""Throughput of the MI355X channelizer path (one JSON line on stdout).

One step = one fe_channelize call over the whole workload: 4 antennas x 2
pols x 2^24 packed 10-bit samples/pol, 4096 channels, 16 taps, int8
channel-major output (all six steps of the path), inputs resident in HBM.
The headline value is the FP32 path; the FP16 and BF16 matrix-core variants
are timed the same way and reported under "variants".
Three input/output buffer sets (about 302 MB each) rotate so no step is
served from the 256 MB Infinity Cache.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Per-kernel durations come from HIP events the library records on its own
stream around each kernel during the timed steps.  The roofline fraction is
the path's algorithmic 2.25 bytes per real sample (1.25 B of packed 10-bit
input, 1 B of int8 output) over the dominant kernel's duration, against the
8 TB/s HBM peak.  The CPU baseline times the FP64 oracle on the host: on the
GPU's share of host cores over the whole workload, and on one thread over a
slice of it.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, published
FP32_PEAK_TFLOPS = 157.3        # MI355X FP32 vector, published
METRIC = "Gsample/s channelized on 1 GPU (FP32 vs FP16-MFMA) + % HBM roofline"
PATH_BYTES_PER_SAMPLE = 2.25    # 10-bit in + int8 complex out, per real sample
# Delay slopes of the timed workloads: the sidereal rate of Sec. 3.3 (below
# 3e-9 samples per sample), so the coarse delay of a call is (nearly)
# constant; the parity tests and the small workload use 1e-5, whose integer
# part steps many times inside one call, and the benchmark reports that
# slope for the large workload as a variant.
SIDEREAL_RATE = 3e-9
DRIFT_RATE = 1e-5


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash() -> str:
    from paper_2303_09886_amd.profsum import source_hash as h
    return h()


def kernel_names(shape: synth.Shape, prec: str, path: str = "split"):
    """The call's kernels by stage, named as rocprofv3 prints them (template
    arguments included), so that the counter summary in profiles/ can be
    looked up: "fir" is the first kernel (the fused unpack + FIR + FFT + post
    kernel where the path is fused), "post" the FFT/post kernel, "turn" the
    corner turn (absent where the FFT/post kernel writes the heaps)."""
    n, T, S = shape.n, shape.taps, shape.spectra_per_heap
    if prec == "fp32":
        tk = next(t for t in (4, 8, 16, 24, 32) if T <= t)
        if path == "fused":
            return {"fir": "pfb_fused_kernel<%d, %d, 0>" % (n, tk), "turn": "corner_turn_kernel"}
        if path == "split_folded":
            return {"fir": "fir_kernel<%d, 0, false>" % tk, "post": "fft_post_heap_kernel<%d, %d>" % (n, 2 if S % 2 == 0 else 1)}
        return {"fir": "fir_kernel<%d, 0, false>" % tk, "post": "fft_post_kernel<%d, 0>" % n, "turn": "corner_turn_kernel"}
    tk = 16 if T <= 16 else 32
    p = 1 if prec == "fp16" else 2
    fir = ("fir_mfma_kernel<%d, %d, %d>" % (tk, p, 0 if prec == "fp16" else 1) if path == "matrix_fir"
           else "fir_kernel<%d, %d, false>" % (next(t for t in (4, 8, 16, 24, 32) if T <= t), 1 if prec == "fp16" else 0))
    if path == "split_folded":
        return {"fir": fir, "post": "fft_mfma_heap_kernel<%d, %d, %d>" % (n, p, 2 if S % 2 == 0 else 1)}
    return {"fir": fir, "post": "fft_mfma_kernel<%d, %d, 0>" % (n, p), "turn": "corner_turn_kernel"}


def measure(fe, shape, w, sets, dev_arrays, prec, steps, warmup, path="auto"):
    """Time `steps` channelize calls of one stream at precision `prec`.

    The wall clock around the timed steps gives the headline rate; the
    library's HIP events, recorded on its own stream around each kernel
    during the same timed steps, give the per-kernel durations."""
    import torch
    N, A, n = shape.samples, shape.antennas, shape.n
    delays, phases, gains = dev_arrays
    st = fe.Stream(n, shape.taps, A, w.weights, N, spectra_per_heap=shape.spectra_per_heap,
                   max_delay=shape.max_delay, precision=prec, path=path)
    path_run = st.schedule()[0]
    log("%s (%s path): warmup %d steps" % (prec, path_run, warmup))
    for i in range(warmup):
        raw, out = sets[i % len(sets)]
        st.channelize(raw, N, delays, phases, gains, out)
    torch.cuda.synchronize()
    log("%s: timing %d steps" % (prec, steps))
    st.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        raw, out = sets[i % len(sets)]
        st.channelize(raw, N, delays, phases, gains, out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fir_ms, post_ms, turn_ms, calls = st.timing_read()
    st.timing(False)
    status = st.status()
    st.close()
    if status != fe.FE_OK:
        log("warning: %s stream status %d" % (prec, status))
    ms_step = (t1 - t0) * 1e3 / steps
    samples = A * 2 * N
    names = kernel_names(shape, prec, path_run)
    avg = {"fir": fir_ms / max(calls, 1), "post": post_ms / max(calls, 1), "turn": turn_ms / max(calls, 1)}
    avg = {k: v for k, v in avg.items() if k in names}
    dom = max(avg, key=avg.get)
    algo = PATH_BYTES_PER_SAMPLE * samples               # algorithmic bytes of one call
    dur_s = avg[dom] * 1e-3
    achieved = algo / dur_s / 1e9
    traffic = stored_traffic(names[dom])
    value = samples / (ms_step * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_over_algorithmic": None if traffic is None else round(traffic / algo, 3),
            "kernel": names[dom], "avg_ms": round(avg[dom], 4), "algorithmic_bytes_per_launch": int(algo),
            "basis": "2.25 B per real input sample (1.25 B packed 10-bit in, 1 B int8 out) x %d samples "
                     "per launch / the kernel's average duration" % samples,
            "call": {"achieved": round(value * PATH_BYTES_PER_SAMPLE, 1),
                     "frac": round(value * PATH_BYTES_PER_SAMPLE / HBM_PEAK_GBS, 4)}}
    kernels = {names[k]: {"avg_ms": round(avg[k], 4), "share_of_call": round(avg[k] / ms_step, 3)}
               for k in avg if avg[k] > 0}
    return {"value": round(value, 2), "ms_per_step": round(ms_step, 4), "path": path_run,
            "hbm_roofline_frac": round(value * PATH_BYTES_PER_SAMPLE / HBM_PEAK_GBS, 4),
            "roofline": roof, "kernels": kernels}


def stored_traffic(kernel: str):
    """HBM traffic per launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def measure_batch(fe, steps: int, warmup: int, tune: bool = True, precision: str = "fp32"):
    """The 16-stream uneven batch: every step runs one call of each stream.
    Timed as one graph launch per step with the launches grouped across the
    members (job-list kernels), as one graph launch per step with every
    member's kernels on a fork stream of its own, and as the same calls
    issued stream after stream on one HIP stream (no overlap).  With
    `precision` fp16 every member runs in FP16 (above 8192 channels: FP16
    storage around the float32 two-level FFT); with bf16 the members of up
    to 8192 channels run in BF16, the larger ones in FP32."""
    import torch
    shapes = synth.BATCH16
    streams, bufs = [], []
    for i, sh in enumerate(shapes):
        w = synth.make_workload(sh, 100 + i, delay_rate=SIDEREAL_RATE)
        M = sh.samples // (2 * sh.n)
        st = fe.Stream(sh.n, sh.taps, 1, w.weights, sh.samples, spectra_per_heap=sh.spectra_per_heap,
                       max_delay=sh.max_delay,
                       precision=precision if (sh.n <= 8192 or precision == "fp16") else "fp32")
        out = torch.empty((1, M // sh.spectra_per_heap, sh.n, sh.spectra_per_heap, 2, 2),
                          dtype=torch.int8, device="cuda")
        b = [torch.from_numpy(w.raw).cuda(), sh.samples, torch.from_numpy(w.delays).cuda(),
             torch.from_numpy(w.phases).cuda(), torch.from_numpy(w.gains).cuda(), out]
        del w
        streams.append(st)
        bufs.append(b)
    torch.cuda.synchronize()
    if tune:
        for st, b in zip(streams, bufs):
            st.autotune(*b, iters=2)
    # the tuned schedule of every member: kernel path and FIR run length /
    # workgroups per CU (two knobs per stream)
    choices = [list(st.schedule()) + [st.fft_parts()] for st in streams]
    total = sum(2 * sh.samples for sh in shapes)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    def sequential():
        for st, b in zip(streams, bufs):
            st.channelize(*b)

    seq_ms = timed(sequential)
    res = {}
    for grouped in (True, False):
        batch = fe.Batch(streams)
        batch.set_grouped(grouped)
        batch.capture(bufs)
        res[grouped] = timed(batch.launch)
        batch.close()
    for st in streams:
        if st.status() != fe.FE_OK:
            log("warning: batch member status %d" % st.status())
        st.close()
    m_ms, g_ms = res[False], res[True]
    return {"value": round(total / (m_ms * 1e-3) / 1e9, 2), "unit": "Gsample/s", "ms_per_step": round(m_ms, 4),
            "issued": "per-member fork streams (the batch default)",
            "grouped_launches_ms_per_step": round(g_ms, 4),
            "grouped_launches_value": round(total / (g_ms * 1e-3) / 1e9, 2),
            "sequential_ms_per_step": round(seq_ms, 4),
            "sequential_value": round(total / (seq_ms * 1e-3) / 1e9, 2),
            "streams": len(shapes), "samples_per_step": total,
            "tuned_schedule": {"knobs": ["path (split|split_folded|fused|matrix_fir)", "fir_batches (FIR run length in batches of "
                                         "spectra, or fused workgroups per CU; 0 = per-launch default)",
                                         "fft_parts (above 8192 channels: workgroups per spectrum of the two-level "
                                         "FFT's post kernel; 0 = per-call default)"],
                               "per_stream": choices},
            "precision": (precision if precision in ("fp32", "fp16")
                          else precision + " (members of up to 8192 channels)"),
            "config": "16 single-antenna streams, channels 1024/4096/8192/32768, taps 8/16/24, "
                      "2^22..2^24 samples/pol each, heaps of 64 spectra, one HIP-graph launch per step; "
                      "grouped: FP32 split-path members through job-list kernels grouped by tap count and "
                      "channel count"}


def measure_service(chunks: int = 24, seed: int = 3):
    """Streaming service: one wide-band antenna (32768 channels, 16 taps),
    chunks of k * 2^20 samples/pol (k uniform in 1..32), already in pinned
    host memory, each with a pinned buffer for its output heaps.  First as a backlog (every chunk waiting at t = 0:
    throughput), then with Poisson arrivals at 70% of that throughput
    (latency under load).  Chunk contents are cut from one generated stretch
    of samples (timing does not depend on them); the rate includes the
    host-to-device and device-to-host copies."""
    from paper_2303_09886_amd import service
    sh = synth.STREAM32K
    unit = sh.samples                                  # 2^20 samples = 32 spectra
    base = synth.make_workload(synth.Shape(n=sh.n, taps=sh.taps, antennas=1, samples=32 * unit,
                                           spectra_per_heap=sh.spectra_per_heap), seed,
                               delay_rate=SIDEREAL_RATE)
    rng = np.random.default_rng(seed)
    ks = rng.integers(1, 33, size=chunks)
    import torch
    # the stretch of samples sits in pinned host memory, as a receive ring
    # would; chunks are views of it
    raw_pin = torch.from_numpy(base.raw[0].copy()).pin_memory()            # [2][32 unit * 5/4]
    d_pin = torch.from_numpy(base.delays[0].copy()).pin_memory()
    p_pin = torch.from_numpy(base.phases[0].copy()).pin_memory()
    g_pin = torch.from_numpy(base.gains[0].copy()).pin_memory()
    spu = unit // (2 * sh.n)                           # spectra per unit

    def requests(rate):
        reqs, t = [], 0.0
        for k in ks:
            N = int(k) * unit
            s0 = int(rng.integers(0, 33 - k))
            if int(k) == 32:
                raw, d, p = raw_pin, d_pin, p_pin
            else:                                      # contiguous copies of the two pols' slices
                raw = torch.empty((2, N * 5 // 4), dtype=torch.uint8).pin_memory()
                raw.copy_(raw_pin[:, s0 * unit * 5 // 4:(s0 + k) * unit * 5 // 4])
                d = d_pin[:, s0 * spu:(s0 + k) * spu].contiguous().pin_memory()
                p = p_pin[:, s0 * spu:(s0 + k) * spu].contiguous().pin_memory()
            if rate:
                t += rng.exponential(N * 2 / rate)
            # the int8 heaps go straight into a pinned buffer of the request
            out = torch.empty(2 * N, dtype=torch.int8).pin_memory()
            reqs.append(service.Request(0, raw, N, d, p, g_pin, arrival=t, out=out))
        return reqs

    # the same chunks already in device memory (input and output): the
    # device side of the service without the host link
    raw_dev, d_dev, p_dev, g_dev = (raw_pin.cuda(), d_pin.cuda(), p_pin.cuda(), g_pin.cuda())

    ks_dev = rng.integers(1, 33, size=64)                 # more chunks: device memory holds them

    def resident(rate):
        reqs, t = [], 0.0
        for k in ks_dev:
            N = int(k) * unit
            s0 = int(rng.integers(0, 33 - k))
            raw = raw_dev[:, s0 * unit * 5 // 4:(s0 + k) * unit * 5 // 4].contiguous()
            d = d_dev[:, s0 * spu:(s0 + k) * spu].contiguous()
            p = p_dev[:, s0 * spu:(s0 + k) * spu].contiguous()
            M = N // (2 * sh.n)
            out = torch.empty((1, M // sh.spectra_per_heap, sh.n, sh.spectra_per_heap, 2, 2), dtype=torch.int8,
                              device="cuda")
            if rate:
                t += rng.exponential(N * 2 / rate)
            reqs.append(service.Request(0, raw, N, d, p, g_dev, arrival=t, out=out))
        torch.cuda.synchronize()
        return reqs

    budget = 4 * service.chunk_device_bytes(sh.n, 32 * unit)
    res = {}
    for kind, make in (("host", requests), ("device_resident", resident)):
        legs = {}
        for mode in ("backlog", "arrivals"):
            svc = service.Service(sh.n, sh.taps, base.weights, feeds=1, max_chunk_samples=32 * unit,
                                  hbm_budget=budget, spectra_per_heap=sh.spectra_per_heap)
            svc.run(make(0), realtime=False)                 # warm-up (allocator, pinned slots)
            rate = 0.7 * legs["backlog"]["gsamples_per_s"] * 1e9 if mode == "arrivals" else 0
            r = svc.run(make(rate), realtime=(mode == "arrivals"))
            svc.close()
            legs[mode] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in r.items()}
            if rate:
                legs[mode]["offered_gsamples_per_s"] = round(rate / 1e9, 3)
        if kind == "host":
            res.update(legs)                                 # backlog / arrivals: host memory in and out
        else:
            res[kind] = legs
    res["config"] = ("1 antenna x 2 pols, 32768 channels (65536-pt real FFT), 16 taps, chunks of k*2^20 "
                     "samples/pol with k uniform in 1..32, heaps of 16 spectra, HBM budget %d MB; backlog and "
                     "arrivals: chunks in pinned host memory, heaps back to pinned host memory; "
                     "device_resident: the same chunks and their outputs in device memory"
                     % (budget >> 20))
    return res


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w: synth.Workload, antennas: int, spectra: int, threads: int, min_seconds: float = 10.0):
    """Time the FP64 oracle on spectra [0, spectra) of the first `antennas`
    antennas (both pols), split over `threads` threads (ctypes releases the
    GIL); the pass is repeated until at least `min_seconds` of wall time have
    been measured.  The rate is channelized real samples per second."""
    import oracle
    oracle.lib()
    s = w.shape
    per = max(1, -(-spectra * antennas // threads))
    tasks = []
    for a in range(antennas):
        for f0 in range(0, spectra, per):
            tasks.append((a, f0, min(spectra, f0 + per)))

    def run(task):
        a, f0, f1 = task
        oracle.channelize(w.raw[a:a + 1], w.total, s.n, s.taps, s.max_delay, w.weights,
                          w.delays[a:a + 1], w.phases[a:a + 1], w.gains[a:a + 1], f0, f1,
                          want=("q",))
        return (f1 - f0) * 2 * 2 * s.n

    samples, passes = 0, 0
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        while True:
            samples += sum(ex.map(run, tasks))
            passes += 1
            dt = time.perf_counter() - t0
            if dt >= min_seconds or passes >= 200:
                break
    return {"value": samples / dt / 1e9, "unit": "Gsample/s", "cores": threads, "kind": "oracle",
            "sample": "%d pass(es) over spectra 0..%d of antennas 0..%d (both pols) of the benchmark "
                      "workload, %d samples in all, FP64 C oracle, %d thread(s)"
                      % (passes, spectra - 1, antennas - 1, samples, threads),
            "seconds": round(dt, 2)}


def measure_small(fe, steps: int, warmup: int):
    """The small workload (1 antenna x 2 pols x 2^20 samples, 1024 channels,
    16 taps): time per call (launch-bound at this size) and its rate."""
    import torch
    sh = synth.SMALL
    w = synth.make_workload(sh, 1)
    M = sh.samples // (2 * sh.n)
    st = fe.Stream(sh.n, sh.taps, sh.antennas, w.weights, sh.samples, spectra_per_heap=sh.spectra_per_heap,
                   max_delay=sh.max_delay)
    args = [torch.from_numpy(a).cuda() for a in (w.raw, w.delays, w.phases, w.gains)]
    out = torch.empty((sh.antennas, M // sh.spectra_per_heap, sh.n, sh.spectra_per_heap, 2, 2),
                      dtype=torch.int8, device="cuda")
    for _ in range(warmup):
        st.channelize(args[0], sh.samples, args[1], args[2], args[3], out)
    torch.cuda.synchronize()
    st.timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        st.channelize(args[0], sh.samples, args[1], args[2], args[3], out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    fir_ms, post_ms, turn_ms, calls = st.timing_read()
    st.timing(False)
    st.close()
    samples = sh.antennas * 2 * sh.samples
    return {"ms_per_call": round(ms, 4), "value": round(samples / (ms * 1e-3) / 1e9, 2), "unit": "Gsample/s",
            "kernel_ms": round((fir_ms + post_ms + turn_ms) / max(calls, 1), 4),
            "config": "1 antenna x 2 pols, 2^20 samples/pol per call, 1024 channels, 16 taps, heaps of 256 "
                      "spectra (the parity workload; its 4.7 MB move in under a microsecond at the HBM "
                      "peak, so the call time is launch latency)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--sets", type=int, default=3, help="rotating input/output buffer sets")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-spectra", type=int, default=None,
                    help="spectra per antenna for the CPU baseline (default: all)")
    ap.add_argument("--variants", default="fp16,bf16,fp16_matrix_fir,fp16_folded,fused,split,drift",
                    help="variants timed beside the FP32 path: fp16, bf16 (DFT stages on the matrix "
                         "cores, vector FIR), fp16_matrix_fir, bf16_matrix_fir (FIR on the matrix cores "
                         "too), fp16_folded, bf16_folded (vector FIR, corner turn folded into the "
                         "matrix-core FFT/post kernel), split, fused, split_folded (the FP32 stream on "
                         "those kernel paths), drift (delays drifting at 1e-5 samples/sample); comma "
                         "list, empty for none")
    ap.add_argument("--no-batch", action="store_true", help="skip the 16-stream batch measurement")
    ap.add_argument("--no-service", action="store_true", help="skip the streaming-service measurement")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 512 MiB device copy (for counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this channelizer build has no multi-GPU path "
              "(antennas are independent; see the sharding notes). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    import paper_2303_09886_amd as fe
    fe.load_library()

    shape = synth.LARGE
    N, A, n, S = shape.samples, shape.antennas, shape.n, shape.spectra_per_heap
    M = N // (2 * n)
    log("generating workload: %s" % (shape,))
    w = synth.make_workload(shape, 2, delay_rate=SIDEREAL_RATE)

    dev = torch.device("cuda:0")
    raw0 = torch.from_numpy(w.raw).to(dev)
    delays = torch.from_numpy(w.delays).to(dev)
    phases = torch.from_numpy(w.phases).to(dev)
    gains = torch.from_numpy(w.gains).to(dev)
    sets = []
    for k in range(args.sets):
        raw = raw0 if k == 0 else torch.roll(raw0, shifts=5 * 977 * k, dims=-1).contiguous()
        out = torch.empty((A, M // S, n, S, 2, 2), dtype=torch.int8, device=dev)
        sets.append((raw, out))
    torch.cuda.synchronize()

    dev_arrays = (delays, phases, gains)
    res = measure(fe, shape, w, sets, dev_arrays, "fp32", args.steps, args.warmup)
    variants = {}
    for prec in args.variants.split(",") if args.variants else []:
        if prec == "drift":
            # the large workload with delays drifting at 1e-5 samples/sample
            wd = synth.make_workload(shape, 2, delay_rate=DRIFT_RATE)
            dd = torch.from_numpy(wd.delays).to(dev)
            variants["fp32_delay_drift_1e-5"] = measure(fe, shape, wd, sets, (dd, phases, gains), "fp32",
                                                        args.steps, args.warmup)
            del wd, dd
            continue
        if prec in ("fp16_matrix_fir", "bf16_matrix_fir"):
            # the reduced-precision stream with its FIR on the matrix cores
            variants[prec] = measure(fe, shape, w, sets, dev_arrays, prec[:4], args.steps, args.warmup,
                                     path="matrix_fir")
            continue
        if prec in ("fp16_folded", "bf16_folded"):
            # the reduced-precision stream with the turn folded into its FFT/post kernel
            variants[prec] = measure(fe, shape, w, sets, dev_arrays, prec[:4], args.steps, args.warmup,
                                     path="split_folded")
            continue
        if prec in ("fused", "split", "split_folded"):
            # the same FP32 stream on another kernel path (fe_stream_set_schedule)
            variants["fp32_" + prec] = measure(fe, shape, w, sets, dev_arrays, "fp32", args.steps, args.warmup,
                                               path=prec)
            continue
        r = measure(fe, shape, w, sets, dev_arrays, prec, args.steps, args.warmup)
        variants[prec + "_mfma"] = r

    batched = None
    if not args.no_batch:
        del sets
        torch.cuda.empty_cache()
        log("batch: 16 uneven streams")
        batched = measure_batch(fe, max(5, args.steps // 5), 2)
        log("batch: 16 uneven streams in FP16")
        batched["fp16"] = measure_batch(fe, max(5, args.steps // 5), 2, precision="fp16")

    streaming = None
    if not args.no_service:
        log("streaming service: 32768 channels")
        streaming = measure_service()

    if args.copy_calibration:
        a = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    small = measure_small(fe, max(20, args.steps), args.warmup)

    cpu = None
    if not args.no_cpu_baseline:
        # the host share of one GPU on these boxes is 16 cores, whatever the
        # machine shows; the single-thread run times a bounded slice
        visible = len(os.sched_getaffinity(0))
        threads = min(16, visible)
        spectra = M if args.cpu_spectra is None else args.cpu_spectra
        log("cpu baseline: oracle over %d spectra x %d antennas, %d threads" % (spectra, A, threads))
        cpu = cpu_baseline(w, A, spectra, threads)
        log("cpu baseline: 1 thread over 96 spectra x 1 antenna")
        one = cpu_baseline(w, 1, min(96, M), 1)
        cpu["single_thread"] = {k: one[k] for k in ("value", "unit", "cores", "sample", "seconds")}
        cpu["cpu_model"] = cpu_model()
        cpu["host_cpus_visible"] = visible

    rec = {
        "metric": METRIC,
        "value": res["value"],
        "unit": "Gsample/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "4 antennas x 2 pols, 2^24 packed 10-bit samples/pol per call, "
                               "4096 channels (8192-pt real FFT), 16-tap PFB, int8 channel-major "
                               "output in heaps of 256 spectra",
                   "antennas": A, "pols": 2, "samples_per_pol": N, "channels": n,
                   "taps": shape.taps, "spectra_per_heap": S, "max_delay": shape.max_delay,
                   "buffer_sets": args.sets},
        "small_workload": small,
        "hbm_roofline_frac": res["hbm_roofline_frac"],
        "roofline": res["roofline"],
        "kernels": res["kernels"],
        "variants": variants,
        "batched": batched,
        "streaming": streaming,
        "cpu_baseline": cpu,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
