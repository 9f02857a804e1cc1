"""Autotuner for batched MAP: how many workgroups (a gang) solve each graph.

The gang size of a graph fixes its rows per workgroup and so its rows per
wavefront (a workgroup has 16 wavefronts).  A policy maps a graph's size to a
gang size.  ``None`` means one workgroup per graph (an ordinary launch that
can be captured in a HIP graph); ``(per_gang, fit)`` means
``gang = clamp(ceil(m / per_gang), 1, cap)``, raised with ``fit`` to
``ceil(n / RES_ROWS)`` so that each workgroup's rows and edges can stay in its
LDS for the whole run (the library falls back to streaming them when they do
not fit).  The tuner times each candidate policy on the actual batch, keeps
the fastest, and caches the choice per device and batch shape in a JSON file
(``$MAPCHECK_TUNE_CACHE``, default ``~/.cache/mapcheck/tune.json``).
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import time

import numpy as np

# Rows one workgroup keeps on chip: 16 wavefronts x 256 rows.
RES_ROWS = 4096
# Upper bound on a gang; the library also clamps to the workgroups of the launch.
CAP = 256
CANDIDATES = (None,
              (1 << 18, False), (1 << 16, False), (1 << 15, False), (1 << 14, False),
              (1 << 18, True), (1 << 16, True), (1 << 15, True), (1 << 14, True))


def policy_name(policy) -> str:
    if policy is None:
        return "one"
    per_gang, fit = policy
    return f"{per_gang}{'+fit' if fit else ''}"


def parse_policy(text: str):
    """Inverse of policy_name: 'one' -> None, '65536+fit' -> (65536, True)."""
    if text == "one":
        return None
    fit = text.endswith("+fit")
    return (int(text[:-4] if fit else text), fit)


def gang_sizes(ns, ms, policy, cap: int = CAP):
    """Gang size per graph for a policy (None -> None, one workgroup each)."""
    if policy is None:
        return None
    per_gang, fit = policy
    out = []
    for n, m in zip(ns, ms):
        g = math.ceil(m / per_gang)
        if fit:
            g = max(g, math.ceil(n / RES_ROWS))
        out.append(int(min(cap, max(1, g))))
    return out


def _cache_path():
    return os.environ.get("MAPCHECK_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mapcheck", "tune.json"))


def _key(device_name, ns, ms):
    h = np.histogram(np.log2(np.maximum(np.asarray(ms, np.float64), 1)), bins=16, range=(0, 32))[0]
    sig = f"{device_name}|{len(ns)}|{int(np.sum(ns))}|{','.join(map(str, h))}"
    return hashlib.sha256(sig.encode()).hexdigest()[:24]


def tune(make_batch, ns, ms, device_name: str, reps: int = 2, use_cache: bool = True, log=None,
         candidates=CANDIDATES):
    """Return (policy, timings) for the batch built by make_batch(gang)."""
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
        p = cache[key]["policy"]
        return (None if p is None else (int(p[0]), bool(p[1]))), cache[key]["timings"]
    timings = {}
    best_policy, best_t = None, float("inf")
    for cand in candidates:
        b = make_batch(gang_sizes(ns, ms, cand))
        b.launch()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            t = time.perf_counter()
            b.launch()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        timings[policy_name(cand)] = best
        if log:
            log(f"[tune] {policy_name(cand)}: {best * 1e3:.2f} ms")
        if best < best_t:
            best_policy, best_t = cand, best
        del b
    if use_cache:
        cache[key] = {"policy": None if best_policy is None else list(best_policy), "timings": timings}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return best_policy, timings


def tune_by(run, candidates=CANDIDATES, log=None):
    """Time run(policy) -> seconds for each candidate policy; return (fastest policy, timings by name)."""
    timings, best, best_t = {}, None, float("inf")
    for cand in candidates:
        t = run(cand)
        timings[policy_name(cand)] = t
        if log:
            log(f"[tune] {policy_name(cand)}: {t * 1e3:.2f} ms")
        if t < best_t:
            best, best_t = cand, t
    return best, timings
