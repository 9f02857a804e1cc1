"""Serving MAP queries with continuous batching on one GPU.

A query is one graph (edge list + accepting flags).  The server:

* admits a query when its device footprint fits the HBM budget, uploads its
  edges from pinned memory and builds its CSR on an upload stream; CSR and
  value state stay resident until the query completes;
* whenever fewer than ``max_inflight`` batches are on the device, launches one
  ``map_detect_batch`` over every admitted query whose CSR is ready, on its own
  stream, so queries that arrive while others run join the next launch and
  their work overlaps with the batch already on the device (workgroups of the
  new launch start as those of the older one retire);
* frees a query's memory when its batch completes and records its latency
  (arrival to result).

All computation runs in the library's HIP kernels; this module only
schedules, allocates and copies.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np
import torch

import paper_0912_2555_amd as mc


def footprint(n: int, m: int) -> int:
    """Device bytes a query holds while admitted (CSR, flags, edge staging, scratch)."""
    return 4 * (n + 1) + 4 * max(m, 1) + n + 8 * max(m, 1) + 5 * n + 2048


@dataclass
class Query:
    qid: int
    n: int
    src: np.ndarray
    dst: np.ndarray
    acc: np.ndarray
    arrival: float = 0.0          # seconds on the server clock
    admitted: float = -1.0
    done: float = -1.0
    result: mc.Result | None = None
    # device state
    csr: mc.Csr | None = None
    acc_dev: torch.Tensor | None = None
    ready: torch.cuda.Event | None = None
    nbytes: int = 0

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class _InFlight:
    queries: list
    batch: mc.Batch
    stream: torch.cuda.Stream
    event: torch.cuda.Event


class Server:
    def __init__(self, hbm_budget: int = 32 << 30, max_inflight: int = 2, gang_policy=None, device="cuda"):
        self.budget = hbm_budget
        self.used = 0
        self.max_inflight = max_inflight
        self.gang_policy = gang_policy      # callable(list of n, list of m) -> gang sizes, or None
        self.device = torch.device(device)
        self.upload = torch.cuda.Stream(device=self.device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(max_inflight)]
        self.free_streams = collections.deque(self.streams)
        self.waiting: collections.deque = collections.deque()   # arrived, not admitted
        self.admitted: list = []                                 # admitted, not launched
        self.inflight: list = []
        self.finished: list = []
        self.build_ws = None
        self.t0 = time.perf_counter()
        self.launches = 0

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # ------------------------------------------------------------ admission
    def arrive(self, q: Query):
        q.arrival = self.now() if q.arrival <= 0 else q.arrival
        self.waiting.append(q)

    def _admit(self):
        while self.waiting:
            q = self.waiting[0]
            need = footprint(q.n, q.m)
            if need > self.budget:
                raise ValueError(f"query {q.qid} needs {need} bytes, more than the whole budget")
            if self.used + need > self.budget:
                return
            self.waiting.popleft()
            self.used += need
            q.nbytes = need
            q.admitted = self.now()
            with torch.cuda.stream(self.upload):
                src = torch.from_numpy(q.src).pin_memory().to(self.device, non_blocking=True)
                dst = torch.from_numpy(q.dst).pin_memory().to(self.device, non_blocking=True)
                q.acc_dev = torch.from_numpy(q.acc).pin_memory().to(self.device, non_blocking=True)
                ws_need = mc.map_workspace_bytes(q.n, q.m)
                if self.build_ws is None or self.build_ws.numel() < ws_need:
                    self.build_ws = torch.empty(ws_need, dtype=torch.uint8, device=self.device)
                q.csr = mc.build_csr(q.n, src, dst, transposed=False, ws=self.build_ws, stream=self.upload,
                                     device=self.device)
                q.ready = torch.cuda.Event()
                q.ready.record(self.upload)
            self.admitted.append(q)

    # ------------------------------------------------------------- launching
    def _launch(self):
        if not self.free_streams:
            return
        ready = [q for q in self.admitted if q.ready.query()]
        if not ready:
            return
        ready.sort(key=lambda q: -q.m)                           # largest first
        self.admitted = [q for q in self.admitted if q not in ready]
        stream = self.free_streams.popleft()
        gang = self.gang_policy([q.n for q in ready], [q.m for q in ready]) if self.gang_policy else None
        with torch.cuda.stream(stream):
            # descriptors, results and workspace are allocated and uploaded on
            # the launch stream, so the launch is ordered after them
            b = mc.Batch([q.csr for q in ready], [q.acc_dev for q in ready], gang=gang, device=self.device)
            b.launch(stream=stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        self.launches += 1
        self.inflight.append(_InFlight(ready, b, stream, ev))

    # ------------------------------------------------------------ completion
    def _complete(self):
        still = []
        for f in self.inflight:
            if f.event.query():
                t = self.now()
                for q, r in zip(f.queries, f.batch.read()):
                    q.result = r
                    q.done = t
                    self.used -= q.nbytes
                    q.csr = None
                    q.acc_dev = None
                    self.finished.append(q)
                self.free_streams.append(f.stream)
            else:
                still.append(f)
        self.inflight = still

    def poll(self):
        self._complete()
        self._admit()
        self._launch()

    def idle(self) -> bool:
        return not (self.waiting or self.admitted or self.inflight)

    def drain(self, timeout: float = 600.0):
        t = time.perf_counter()
        while not self.idle():
            self.poll()
            if time.perf_counter() - t > timeout:
                raise TimeoutError("server did not drain")
            time.sleep(50e-6)


def run_stream(queries, qps: float, server: Server, gaps=None):
    """Replay a Poisson arrival stream (unit-mean gaps scaled by 1/qps) through the server."""
    gaps = gaps if gaps is not None else np.random.default_rng(0).exponential(1.0, len(queries))
    arrivals = np.cumsum(np.asarray(gaps, np.float64) / qps)
    start = server.now()
    i = 0
    while i < len(queries) or not server.idle():
        t = server.now() - start
        while i < len(queries) and arrivals[i] <= t:
            queries[i].arrival = start + arrivals[i]
            server.arrive(queries[i])
            i += 1
        server.poll()
        time.sleep(20e-6)
    span = server.now() - start
    lat = np.array([q.latency for q in queries])
    return {"graphs_per_s": len(queries) / span, "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "span_s": span, "launches": server.launches}


def run_serial(queries, qps: float, gaps=None, device="cuda"):
    """The baseline: the same arrival stream served one query at a time with map_detect."""
    dev = torch.device(device)
    gaps = gaps if gaps is not None else np.random.default_rng(0).exponential(1.0, len(queries))
    arrivals = np.cumsum(np.asarray(gaps, np.float64) / qps)
    t0 = time.perf_counter()
    lat = []
    results = []
    for q, a in zip(queries, arrivals):
        now = time.perf_counter() - t0
        if now < a:
            time.sleep(a - now)
        csr = mc.build_csr(q.n, q.src, q.dst, transposed=False, device=dev)
        out = mc.detect(csr, q.acc)
        results.append(out.result)
        lat.append(time.perf_counter() - t0 - a)
    span = time.perf_counter() - t0
    lat = np.array(lat)
    return {"graphs_per_s": len(queries) / span, "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "span_s": span}, results
