"""Streaming channelizer service: a request loop over the C ABI.

Feeds (single-antenna, dual-polarization streams) send chunks of packed
samples of any whole number of heaps, arriving over time.  Each feed has one
``fe_stream``: its PFB tail (the last 2n(T-1)+D_max samples), its delay
handling and its sample count stay on the device between chunks (Secs. 3.1
and 3.3), so a feed's chunks are processed in arrival order.

The loop is continuously batched: a chunk is admitted as soon as the device
memory it needs (its input, metadata and output buffers) fits the HBM budget
next to the work already in flight; it is then copied to the device and
channelized on its feed's own HIP stream.  Different feeds' chunks therefore
run concurrently on the GPU, chunks that arrive while others run join as
memory frees up, and a feed's chunks queue behind each other on its stream.
Completion is event-driven: a thread per feed blocks on its oldest chunk's
HIP event and releases the chunk's memory; the int8 heaps come back to
pinned host memory, or stay on the device when the request brought device
buffers (input and output already in HBM: the device-side figures).
Latency = completion time - arrival time.

All channelizer arithmetic runs in the library's HIP kernels; this module
schedules, moves buffers and keeps time.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Dict, List, Optional

import numpy as np

from . import fengine


def chunk_device_bytes(n_channels: int, n_samples: int) -> int:
    """Device bytes one chunk holds while in flight: packed input of both
    pols, delays and phases, gains, int8 output."""
    M = n_samples // (2 * n_channels)
    return 2 * n_samples * 5 // 4 + 2 * 2 * M * 8 + 2 * n_channels * 8 + 2 * n_samples


@dataclasses.dataclass
class Request:
    """One chunk of one feed.

    raw     uint8 [2][N*5/4] packed 10-bit samples (host: a numpy array, or
            a pinned torch tensor, which is copied to the device directly;
            or, with every other buffer including ``out``, a device tensor:
            the chunk is then channelized in place, nothing is copied)
    delays  float64 [2][M], phases float64 [2][M]  (M = N / 2n)
    gains   float32 [2][n][2]
    arrival seconds on the loop's clock (0 = loop start)
    out     optional pinned torch int8 tensor of at least 2N elements: the
            heaps are copied from the device straight into it; otherwise they
            pass through a pinned staging slot and ``out`` becomes a numpy
            copy, [1][M/S][n][S][2][2]
    """
    feed: int
    raw: np.ndarray
    n_samples: int
    delays: np.ndarray
    phases: np.ndarray
    gains: np.ndarray
    arrival: float = 0.0
    out: Optional[object] = None
    # filled in by the service
    admitted: float = -1.0
    done: float = -1.0

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Service:
    """``feeds`` streams of one shape (n channels, T taps) sharing a GPU and
    an HBM budget (bytes) for in-flight chunks."""

    def __init__(self, n_channels: int, taps: int, weights, feeds: int, max_chunk_samples: int,
                 hbm_budget: int, spectra_per_heap: int = 16, max_delay: int = 128,
                 precision: str = "fp32", host_slots: int = 8):
        import torch
        self.torch = torch
        self.n, self.taps, self.S = n_channels, taps, spectra_per_heap
        self.budget = int(hbm_budget)
        # per feed: the compute stream (the feed's fe_stream), and copy
        # streams in and out, so a chunk's transfers overlap its neighbours'
        # kernels; all at default priority
        self.hip = [torch.cuda.Stream() for _ in range(feeds)]
        self.h2d = [torch.cuda.Stream() for _ in range(feeds)]
        self.d2h = [torch.cuda.Stream() for _ in range(feeds)]
        self.streams = [fengine.Stream(n_channels, taps, 1, weights, max_chunk_samples,
                                       spectra_per_heap=spectra_per_heap, max_delay=max_delay,
                                       hip_stream=self.hip[f], precision=precision)
                        for f in range(feeds)]
        self.max_chunk = max_chunk_samples
        # pinned host staging, reused: one slot per chunk in flight
        self.slots = []
        self.host_slots = host_slots

    def _slot(self):
        torch = self.torch
        if self.slots:
            return self.slots.pop()
        Mx = self.max_chunk // (2 * self.n)
        return {"raw": torch.empty(2 * self.max_chunk * 5 // 4, dtype=torch.uint8, pin_memory=True),
                "d": torch.empty(2 * Mx, dtype=torch.float64, pin_memory=True),
                "p": torch.empty(2 * Mx, dtype=torch.float64, pin_memory=True),
                "g": torch.empty(2 * self.n * 2, dtype=torch.float32, pin_memory=True),
                "out": torch.empty(2 * self.max_chunk, dtype=torch.int8, pin_memory=True)}

    def chunk_bytes(self, n_samples: int) -> int:
        return chunk_device_bytes(self.n, n_samples)

    def _start(self, r: Request, now: float, slot):
        torch = self.torch
        f = r.feed
        N = r.n_samples
        M = N // (2 * self.n)
        nb = 2 * N * 5 // 4
        if self._resident(r):
            # everything already in device memory: the call alone
            self.streams[f].channelize(r.raw, N, r.delays, r.phases, r.gains, r.out)
            ev = torch.cuda.Event()
            ev.record(self.hip[f])
            r.admitted = now
            return {"req": r, "event": ev, "keep": None, "slot": slot, "own": True,
                    "shape": tuple(r.out.shape), "bytes": self.chunk_bytes(N)}
        # host side: chunks that already sit in pinned host memory (torch
        # tensors, as a receive ring would hold them) are copied straight to
        # the device; others go through the pinned staging slot first
        def staged(a, name, count, dtype):
            if isinstance(a, torch.Tensor) and a.is_pinned():
                return a.reshape(-1)[:count]
            slot[name][:count].copy_(torch.from_numpy(np.ascontiguousarray(a, dtype=dtype).reshape(-1)))
            return slot[name][:count]

        src = [staged(r.raw, "raw", nb, np.uint8), staged(r.delays, "d", 2 * M, np.float64),
               staged(r.phases, "p", 2 * M, np.float64), staged(r.gains, "g", 4 * self.n, np.float32)]
        with torch.cuda.stream(self.h2d[f]):
            raw, d, ph, g = [x.to("cuda", non_blocking=True) for x in src]
            out = torch.empty((1, M // self.S, self.n, self.S, 2, 2), dtype=torch.int8, device="cuda")
            ev_in = torch.cuda.Event()
            ev_in.record(self.h2d[f])
        self.hip[f].wait_event(ev_in)
        self.streams[f].channelize(raw, N, d, ph, g, out)         # enqueued on self.hip[f]
        ev_k = torch.cuda.Event()
        ev_k.record(self.hip[f])
        self.d2h[f].wait_event(ev_k)
        own = isinstance(r.out, torch.Tensor) and r.out.is_pinned() and r.out.numel() >= 2 * N
        dst = r.out.reshape(-1)[:2 * N] if own else slot["out"][:2 * N]
        with torch.cuda.stream(self.d2h[f]):
            dst.copy_(out.reshape(-1).view(dst.dtype), non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.d2h[f])
        r.admitted = now
        # device buffers stay referenced until the event has passed
        return {"req": r, "event": ev, "keep": (raw, d, ph, g, out), "slot": slot, "own": own,
                "shape": tuple(out.shape), "bytes": self.chunk_bytes(N)}

    def _resident(self, r: Request) -> bool:
        """A request whose buffers are all device tensors (output included)."""
        torch = self.torch
        return all(isinstance(a, torch.Tensor) and a.is_cuda for a in (r.raw, r.delays, r.phases, r.gains, r.out))

    def run(self, requests: List[Request], realtime: bool = True) -> Dict:
        """Serve ``requests`` (sorted by arrival).  ``realtime``: admit a
        request no earlier than its arrival time; otherwise all arrive at 0.
        Returns throughput and latency statistics; outputs land in req.out.

        Completion is event-driven: one thread per feed blocks on the HIP
        event of its feed's oldest chunk in flight (a feed's chunks finish in
        order) and then releases the chunk's memory; the admitting loop
        sleeps on a condition variable until a chunk arrives or memory frees
        up."""
        import threading
        import queue
        for r in requests:
            if r.n_samples % (2 * self.n * self.S) or r.n_samples > self.max_chunk:
                raise ValueError("chunk of %d samples does not fit the service" % r.n_samples)
            if self.chunk_bytes(r.n_samples) > self.budget:
                raise ValueError("chunk larger than the HBM budget")
        pending = sorted(requests, key=lambda r: r.arrival)
        if not realtime:
            for r in pending:
                r.arrival = 0.0
        cond = threading.Condition()
        state = {"used": 0, "inflight": 0, "peak": 0, "error": None}
        queues = [queue.Queue() for _ in self.streams]
        t0 = time.perf_counter()

        def complete(f):
            while True:
                job = queues[f].get()
                if job is None:
                    return
                try:
                    job["event"].synchronize()                 # blocks without the interpreter lock
                    r = job["req"]
                    r.done = time.perf_counter() - t0
                    if not job["own"]:
                        k = 2 * r.n_samples
                        r.out = job["slot"]["out"][:k].numpy().reshape(job["shape"]).copy()
                except Exception as e:                         # reported by run()
                    state["error"] = e
                with cond:
                    if job["slot"] is not None:
                        self.slots.append(job["slot"])
                    state["used"] -= job["bytes"]
                    state["inflight"] -= 1
                    cond.notify_all()

        threads = [threading.Thread(target=complete, args=(f,), daemon=True) for f in range(len(self.streams))]
        for t in threads:
            t.start()
        try:
            for r in pending:
                need = self.chunk_bytes(r.n_samples)
                resident = self._resident(r)
                with cond:
                    while True:
                        if state["error"] is not None:
                            raise state["error"]
                        now = time.perf_counter() - t0
                        if r.arrival > now:
                            cond.wait(timeout=r.arrival - now)
                            continue
                        if state["used"] + need > self.budget or (not resident and state["inflight"] >= self.host_slots):
                            cond.wait()
                            continue
                        state["used"] += need
                        state["inflight"] += 1
                        state["peak"] = max(state["peak"], state["used"])
                        break
                job = self._start(r, time.perf_counter() - t0, None if resident else self._slot_locked(cond))
                queues[r.feed].put(job)
        finally:
            for q in queues:
                q.put(None)
            for t in threads:
                t.join()
        if state["error"] is not None:
            raise state["error"]
        wall = max(r.done for r in requests) if requests else 0.0
        lat = np.array([r.latency for r in requests]) * 1e3
        # latency per 2^20 samples of the chunk: chunks of different sizes
        # take different times even alone, this spread is the scheduling's
        per_m = lat / np.array([r.n_samples / float(1 << 20) for r in requests])
        samples = 2 * sum(r.n_samples for r in requests)
        for st in self.streams:
            if st.status() != fengine.FE_OK:
                raise fengine.FEngineError(st.status(), "service stream")
        return {"chunks": len(requests), "samples": samples, "seconds": wall,
                "gsamples_per_s": samples / wall / 1e9,
                "latency_ms_p50": float(np.percentile(lat, 50)),
                "latency_ms_p99": float(np.percentile(lat, 99)),
                "latency_ms_max": float(lat.max()),
                "latency_ms_per_2e20_samples_p50": float(np.percentile(per_m, 50)),
                "latency_ms_per_2e20_samples_p99": float(np.percentile(per_m, 99)),
                "peak_inflight_bytes": state["peak"]}

    def _slot_locked(self, cond):
        with cond:
            return self._slot()

    def close(self):
        for st in self.streams:
            st.close()
        self.streams = []
