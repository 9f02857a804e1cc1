"""Detection on a growing graph.

The paper's tool builds the graph's matrix in one thread while a second thread
repeatedly runs the accepting-cycle detection on the part built so far, so a
cycle present in that part is reported before the whole state space exists
(Section 2); it also keeps only the states of components that contain
accepting states.  Here the graph arrives as an edge stream already resident
in device memory (in generation order), and ``detect_stream`` runs, for each
prefix of 1/chunks, 2/chunks, ... of the stream, the library's CSR build, its
relevance pruning (``map_trim``: vertices that can lie on no cycle lose their
accepting flag) and its MAP outer loop (``map_detect``), stopping at the first
prefix that holds an accepting cycle.  A cycle in a prefix is a cycle of every
longer prefix, so the verdict found early is final; a prefix without one says
nothing about the rest.

All computation runs in the library's HIP kernels; this module only slices
the stream and reads each prefix's result.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import torch

import paper_0912_2555_amd as mc


@dataclass
class Prefix:
    edges: int            # edges of the stream in this prefix
    found: int
    witness: int
    iterations: int
    kept: int             # vertices kept by the pruning (-1 without pruning)
    accepting_kept: int   # accepting vertices kept (-1 without pruning)
    sweeps: int           # propagation sweeps of the detection
    ms: float             # wall time of build + pruning + detection for this prefix
    build_ms: float       # device time of each stage (HIP events on the current stream)
    trim_ms: float
    detect_ms: float


@dataclass
class StreamOut:
    found: int
    witness: int
    edges_at_verdict: int          # prefix length when the loop stopped
    total_ms: float
    prefixes: list = field(default_factory=list)


def detect_stream(n: int, src: torch.Tensor, dst: torch.Tensor, accepting: torch.Tensor, chunks: int = 16,
                  prune: bool = True, ws: torch.Tensor | None = None) -> StreamOut:
    """Run build / prune / detect on growing prefixes of a device-resident edge stream (1-based ids)."""
    if chunks < 1:
        raise ValueError("chunks must be >= 1")
    dev = src.device
    m = int(src.numel())
    acc = accepting.to(dev, dtype=torch.uint8).contiguous()
    if ws is None:
        ws = mc.workspace(n, m, device=dev)
    out = StreamOut(0, 0, 0, 0.0)
    t_all = time.perf_counter()
    stream = torch.cuda.current_stream(dev)
    for c in range(1, chunks + 1):
        pm = m * c // chunks
        if pm == 0 and c < chunks:
            continue
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        t = time.perf_counter()
        ev[0].record(stream)
        csr = mc.build_csr(n, src[:pm], dst[:pm], transposed=prune, ws=ws, device=dev)
        ev[1].record(stream)
        kept = acc_kept = -1
        acc_use = acc
        if prune:
            tr = mc.trim(csr, acc, ws=ws)
            if tr.status != mc.MAP_OK:
                raise mc.MapError(tr.status, "map_trim (device)")
            kept, acc_kept, acc_use = tr.kept, tr.accepting_kept, tr.accepting
        ev[2].record(stream)
        r = mc.detect(csr, acc_use, ws=ws).result
        ev[3].record(stream)
        if r.status != mc.MAP_OK:
            raise mc.MapError(r.status, "map_detect (device)")
        ms = (time.perf_counter() - t) * 1e3
        ev[3].synchronize()
        out.prefixes.append(Prefix(pm, r.found, r.witness, r.iterations, kept, acc_kept, r.sweeps, ms,
                                   ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]),
                                   ev[2].elapsed_time(ev[3])))
        out.edges_at_verdict = pm
        if r.found:
            out.found, out.witness = 1, r.witness
            break
    out.total_ms = (time.perf_counter() - t_all) * 1e3
    return out
