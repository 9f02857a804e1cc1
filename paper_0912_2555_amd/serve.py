"""Serving MAP queries with continuous batching on one GPU.

A query is one graph: an edge list and accepting flags in pinned host memory
(a receive buffer; other host arrays are pinned on arrival).  The server keeps
one ``map_engine`` running on the device for its whole life and:

* admits a query when its device footprint (CSR and scratch) fits the HBM
  budget: the budget is one arena allocated up front and carved per query by
  a first-fit allocator, so nothing is allocated while the engine runs;
* posts the admitted query to the running engine at once: free workgroups
  pick it up while the engine keeps working on earlier queries, read its edge
  list and flags straight from pinned host memory, build its CSR into the
  arena block and run the MAP loop (no copy or launch runs beside the engine);
* frees the arena block when the engine reports the query finished, and
  records its latency (arrival to result).

All computation runs in the library's HIP kernels; this module only
schedules, allocates and pins.
"""
from __future__ import annotations

import bisect
import collections
import time
from dataclasses import dataclass

import numpy as np
import torch

import paper_0912_2555_amd as mc

_ALIGN = 256


def _al(x: int) -> int:
    return (x + _ALIGN - 1) & ~(_ALIGN - 1)


def _layout(n: int, m: int):
    """Byte offsets of a query's device buffers inside its arena block, and the block size."""
    off, out = 0, {}
    for name, nbytes in (("row_ptr", 4 * (n + 1)), ("col", 4 * max(m, 1)),
                         ("scratch", mc.map_job_scratch_bytes(n, m))):
        out[name] = (off, nbytes)
        off += _al(nbytes)
    return out, off


def footprint(n: int, m: int) -> int:
    """Device bytes a query holds while admitted (CSR and scratch)."""
    return _layout(n, m)[1]


class Arena:
    """First-fit allocator of byte ranges in [0, size), with coalescing frees."""

    def __init__(self, size: int):
        self.size = size
        self.free_off = [0]          # sorted offsets of free ranges
        self.free_len = {0: size}

    def alloc(self, nbytes: int):
        nbytes = _al(nbytes)
        for off in self.free_off:
            ln = self.free_len[off]
            if ln >= nbytes:
                i = bisect.bisect_left(self.free_off, off)
                del self.free_off[i]
                del self.free_len[off]
                if ln > nbytes:
                    bisect.insort(self.free_off, off + nbytes)
                    self.free_len[off + nbytes] = ln - nbytes
                return off
        return None

    def free(self, off: int, nbytes: int):
        nbytes = _al(nbytes)
        i = bisect.bisect_left(self.free_off, off)
        # merge with the next range
        if i < len(self.free_off) and self.free_off[i] == off + nbytes:
            nbytes += self.free_len.pop(self.free_off[i])
            del self.free_off[i]
        # merge with the previous range
        if i > 0 and self.free_off[i - 1] + self.free_len[self.free_off[i - 1]] == off:
            self.free_len[self.free_off[i - 1]] += nbytes
            return
        self.free_off.insert(i, off)
        self.free_len[off] = nbytes

    def free_bytes(self) -> int:
        return sum(self.free_len.values())


def _pinned(x, dtype):
    """x as a device or pinned host tensor (a pinned copy of anything else)."""
    if isinstance(x, torch.Tensor) and (x.is_cuda or x.is_pinned()):
        return x
    t = x if isinstance(x, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(x, dtype=dtype))
    return t.pin_memory()


@dataclass
class Query:
    qid: int
    n: int
    src: object                  # int32[m] edge sources (pinned host tensor; other arrays are pinned on arrival)
    dst: object                  # int32[m]
    acc: object                  # uint8[n]
    arrival: float = 0.0         # seconds on the server clock
    admitted: float = -1.0
    started: float = -1.0        # posted to the engine
    done: float = -1.0
    result: mc.Result | None = None
    # server state
    off: int = -1
    nbytes: int = 0
    bufs: dict | None = None
    slot: int = -1

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Server:
    """Continuous-batching MAP server on one running map_engine."""

    def __init__(self, hbm_budget: int = 32 << 30, gang_policy=None, max_jobs: int = 1024, workgroups: int = 0,
                 idle_seconds: float = 60.0, device="cuda", flags: int = 0):
        self.device = torch.device(device)
        self.budget = hbm_budget
        self.gang_policy = gang_policy      # callable(list of n, list of m) -> gang sizes, or None (1 each)
        self.arena_mem = torch.empty(hbm_budget, dtype=torch.uint8, device=self.device)
        self.arena = Arena(hbm_budget)
        torch.cuda.synchronize(self.device)
        # flags: MAP_FLAG_DIRECTION runs every query with filtered sweeps and the
        # direction switch (its scratch already has room for the transposed CSR)
        self.flags = flags
        self.engine = mc.Engine(max_jobs=max_jobs, workgroups=workgroups, idle_seconds=idle_seconds, flags=flags,
                                device=self.device)
        self.waiting: collections.deque = collections.deque()   # arrived, not admitted
        self.admitted: collections.deque = collections.deque()  # admitted, not yet taken by the engine
        self.running: dict = {}                                  # slot -> query
        self.finished: list = []
        self.t0 = time.perf_counter()
        self.submitted = 0
        self.max_running = 0                                     # most queries on the engine at once

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def used(self) -> int:
        return self.budget - self.arena.free_bytes()

    # ------------------------------------------------------------ admission
    def arrive(self, q: Query):
        if footprint(q.n, q.m) > self.budget:
            raise ValueError(f"query {q.qid} needs {footprint(q.n, q.m)} bytes, more than the whole budget")
        q.src, q.dst, q.acc = _pinned(q.src, np.int32), _pinned(q.dst, np.int32), _pinned(q.acc, np.uint8)
        q.arrival = self.now() if q.arrival <= 0 else q.arrival
        self.waiting.append(q)

    def _admit(self):
        while self.waiting:
            q = self.waiting[0]
            lay, need = _layout(q.n, q.m)
            off = self.arena.alloc(need)
            if off is None:
                return
            self.waiting.popleft()
            q.off, q.nbytes, q.admitted = off, need, self.now()
            b = {k: self.arena_mem[off + o:off + o + ln] for k, (o, ln) in lay.items()}
            b["row_ptr"] = b["row_ptr"].view(torch.int32)
            b["col"] = b["col"].view(torch.int32)
            q.bufs = b
            self.admitted.append(q)

    # ------------------------------------------------------------ submission
    def _submit(self):
        if not self.admitted:
            return
        batch = list(self.admitted)
        gangs = self.gang_policy([q.n for q in batch], [q.m for q in batch]) if self.gang_policy else None
        for i, q in enumerate(batch):
            b, m = q.bufs, q.m
            slot = self.engine.submit(q.n, q.src if m else None, q.dst if m else None, b["row_ptr"],
                                      b["col"], q.acc, b["scratch"], gang=gangs[i] if gangs else 1, tag=q.qid)
            if slot is None:                      # engine full: retry on the next poll
                return
            self.admitted.popleft()
            q.slot, q.started = slot, self.now()
            self.running[slot] = q
            self.submitted += 1
            self.max_running = max(self.max_running, len(self.running))

    # ------------------------------------------------------------ completion
    def _complete(self):
        for slot in list(self.running):
            r = self.engine.poll(slot)
            if r is None:
                continue
            q = self.running.pop(slot)
            q.result, q.done = r, self.now()
            self.arena.free(q.off, q.nbytes)
            q.bufs = None
            self.finished.append(q)

    def poll(self):
        self._complete()
        self._admit()
        self._submit()

    def idle(self) -> bool:
        return not (self.waiting or self.admitted or self.running)

    def drain(self, timeout: float = 600.0):
        t = time.perf_counter()
        while not self.idle():
            self.poll()
            if time.perf_counter() - t > timeout:
                raise TimeoutError("server did not drain")
            time.sleep(20e-6)

    def close(self):
        self.engine.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _stats(queries, span):
    lat = np.array([q.latency for q in queries])
    return {"graphs_per_s": len(queries) / span, "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3), "span_s": span}


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
        time.sleep(10e-6)
    out = _stats(queries, server.now() - start)
    out["jobs"] = server.submitted
    return out


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
        src = _pinned(q.src, np.int32).to(dev, non_blocking=True)
        dst = _pinned(q.dst, np.int32).to(dev, non_blocking=True)
        acc = _pinned(q.acc, np.uint8).to(dev, non_blocking=True)
        csr = mc.build_csr(q.n, src, dst, transposed=False, device=dev)
        out = mc.detect(csr, acc)
        results.append(out.result)
        lat.append(time.perf_counter() - t0 - a)
    span = time.perf_counter() - t0
    lat = np.array(lat)
    return {"graphs_per_s": len(queries) / span, "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "span_s": span}, results
