"""Autotuner for batched MAP: how many workgroups (a gang) solve each graph.

The gang size of a graph fixes its rows per workgroup and so its rows per
wavefront (a workgroup has 16 wavefronts).  A policy maps a graph's edge
count to a gang size: ``gang = clamp(ceil(m / per_gang), 1, cap)``, with
``per_gang = None`` meaning one workgroup per graph (an ordinary launch that
can be captured in a HIP graph).  The tuner times each candidate policy on the
actual batch, keeps the fastest, and caches the choice per device and batch
shape in a JSON file (``$MAPCHECK_TUNE_CACHE``, default
``~/.cache/mapcheck/tune.json``).
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import time

import numpy as np

CANDIDATES = (None, 1 << 19, 1 << 18, 1 << 17, 1 << 16, 1 << 15)
CAP = 64


def gang_sizes(ms, per_gang, cap: int = CAP):
    """Gang size per graph for a policy (None -> all ones)."""
    if per_gang is None:
        return None
    return [int(min(cap, max(1, math.ceil(m / per_gang)))) for m in ms]


def _cache_path():
    return os.environ.get("MAPCHECK_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mapcheck", "tune.json"))


def _key(device_name, ns, ms):
    h = np.histogram(np.log2(np.maximum(np.asarray(ms, np.float64), 1)), bins=16, range=(0, 32))[0]
    sig = f"{device_name}|{len(ns)}|{int(np.sum(ns))}|{','.join(map(str, h))}"
    return hashlib.sha256(sig.encode()).hexdigest()[:24]


def tune(make_batch, ns, ms, device_name: str, reps: int = 2, use_cache: bool = True, log=None):
    """Return (per_gang, timings) for the batch built by make_batch(gang)."""
    import torch
    key = _key(device_name, ns, ms)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        return cache[key]["per_gang"], cache[key]["timings"]
    timings = {}
    for cand in CANDIDATES:
        b = make_batch(gang_sizes(ms, cand))
        b.launch()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            t = time.perf_counter()
            b.launch()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        timings[str(cand)] = best
        if log:
            log(f"[tune] per_gang={cand}: {best * 1e3:.2f} ms")
        del b
    best_key = min(timings, key=timings.get)
    per_gang = None if best_key == "None" else int(best_key)
    if use_cache:
        cache[key] = {"per_gang": per_gang, "timings": timings}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return per_gang, timings
