"""Autotuner for batched MAP: how each graph of a batch is solved.

Two knobs per graph class:

- the gang: how many workgroups solve a graph.  It fixes the graph's rows per
  workgroup and so its rows per wavefront (a workgroup has 16 wavefronts).  A
  gang policy maps a graph's size to a gang size.  ``None`` means one
  workgroup per graph (an ordinary launch); ``(per_gang, fit)`` means
  ``gang = clamp(ceil(m / per_gang), 1, cap)``, raised with ``fit`` to
  ``ceil(n / RES_ROWS)`` so that each workgroup's rows and edges can stay in
  its LDS for the whole run (the library streams them when they do not fit).
  Both kinds of launch can be captured in a HIP graph.
- the per-graph options (map_graph_desc.options): the fixpoint control of a
  multi-workgroup gang (asynchronous sweeps or a barrier after every sweep),
  whether its CSR is streamed instead of staged on chip, whether streamed
  sweeps gather only from rows that grew (filtered sweeps) and switch to push
  rounds over the transposed CSR on small frontiers, and the long-row
  threshold above which a streamed row is folded by a whole wavefront.  An
  option rule maps a graph's class -- its gang size, n and largest out-degree
  -- to options.

The tuner times the gang policies on the actual batch, then the option rules
on the fastest gang policy, then (if a rule won) the gang policies again under
that rule, keeps the fastest pair, and caches it per device
and batch shape in a JSON file (``$MAPCHECK_TUNE_CACHE``, default
``~/.cache/mapcheck/tune.json``).  No knob changes a result.
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


# map_graph_desc.options bits (include/mapcheck.h)
GRAPH_SYNC_SWEEPS = 0x10000
GRAPH_STREAM = 0x20000
GRAPH_FILTER = 0x40000
GRAPH_DIRECTION = 0x80000
HUB_NEVER = 0xFFFF
# Option rules: name -> options(gang, n, max_degree).
OPTION_RULES = {
    "default": lambda gang, n, dmax: 0,
    "sync-gangs": lambda gang, n, dmax: GRAPH_SYNC_SWEEPS if gang > 1 else 0,
    "sync-small-gangs": lambda gang, n, dmax: GRAPH_SYNC_SWEEPS if 1 < gang <= 8 else 0,
    "stream-single": lambda gang, n, dmax: GRAPH_STREAM if gang == 1 else 0,
    "hub8": lambda gang, n, dmax: 8 if dmax > 8 else 0,
    "hub-never": lambda gang, n, dmax: HUB_NEVER,
    "filter-gangs": lambda gang, n, dmax: GRAPH_FILTER if gang > 1 else 0,
    "filter-all": lambda gang, n, dmax: GRAPH_FILTER,
    # Direction switch (push rounds on small frontiers): needs each graph's
    # transposed CSR, otherwise the option is ignored.
    "direction-gangs": lambda gang, n, dmax: GRAPH_FILTER | GRAPH_DIRECTION if gang > 1 else 0,
    "direction-all": lambda gang, n, dmax: GRAPH_FILTER | GRAPH_DIRECTION,
}


def graph_options(rule: str, gangs, ns, dmaxs):
    """Per-graph options of an option rule (gangs None: one workgroup each)."""
    f = OPTION_RULES[rule]
    gangs = [1] * len(ns) if gangs is None else gangs
    return [int(f(g, n, d)) for g, n, d in zip(gangs, ns, dmaxs)]


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


def tune_knobs(make_batch, ns, ms, dmaxs, device_name: str, reps: int = 2, use_cache: bool = True, log=None,
               gang_candidates=CANDIDATES, rules=tuple(OPTION_RULES)):
    """Both knobs: the gang policy (options at their defaults), then the option
    rule on the fastest gang policy, then (when a rule other than the default
    won) the gang policies again under that rule.  make_batch(gangs, options)
    builds the batch.  Returns ({"gang": policy, "options": rule}, timings by
    name)."""
    import torch
    key = "knobs|" + _key(device_name, ns, ms) + "|" + str(int(np.max(dmaxs)) if len(dmaxs) else 0)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        e = cache[key]
        p = e["gang"]
        return {"gang": None if p is None else (int(p[0]), bool(p[1])), "options": e["options"]}, e["timings"]

    def time_batch(gangs, options):
        b = make_batch(gangs, options)
        b.launch()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            t = time.perf_counter()
            b.launch()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        del b
        return best

    timings = {}
    best_gang, best_t = None, float("inf")
    for cand in gang_candidates:
        t = time_batch(gang_sizes(ns, ms, cand), None)
        timings["gang:" + policy_name(cand)] = t
        if log:
            log(f"[tune] gang {policy_name(cand)}: {t * 1e3:.2f} ms")
        if t < best_t:
            best_gang, best_t = cand, t
    gangs = gang_sizes(ns, ms, best_gang)
    best_rule = "default"
    timings["options:default"] = best_t
    for rule in rules:
        if rule == "default":
            continue
        t = time_batch(gangs, graph_options(rule, gangs, ns, dmaxs))
        timings["options:" + rule] = t
        if log:
            log(f"[tune] options {rule}: {t * 1e3:.2f} ms")
        if t < best_t:
            best_rule, best_t = rule, t
    if best_rule != "default":
        # The gang policies again, under the chosen option rule (an option such
        # as the direction switch changes which gang size pays); the first
        # stage's winner was timed under the rule already.
        first = best_gang
        for cand in gang_candidates:
            if cand == first:
                continue
            g2 = gang_sizes(ns, ms, cand)
            t = time_batch(g2, graph_options(best_rule, g2, ns, dmaxs))
            timings["gang:" + policy_name(cand) + "|" + best_rule] = t
            if log:
                log(f"[tune] gang {policy_name(cand)} with {best_rule}: {t * 1e3:.2f} ms")
            if t < best_t:
                best_gang, best_t = cand, t
    choice = {"gang": best_gang, "options": best_rule}
    if use_cache:
        cache[key] = {"gang": None if best_gang is None else list(best_gang), "options": best_rule,
                      "timings": timings}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return choice, timings


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
