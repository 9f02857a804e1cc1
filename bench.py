"""Benchmark: MAP accepting-cycle detection on one MI355X.

A step is one pass of the whole hot path over the workload: build the CSR of
the resident edge list on the device (pull and transposed), then the MAP outer
loop to its exit (map_detect).  Inputs are generated once, uploaded, and stay
in HBM; the timed region starts with them resident.

Default workload: the state-space-shaped graph with 2^20 vertices in BFS order
(out-degree 1+Poisson(3), 80% local / 20% uniform, 90% forward / 10% back
edges, 1% accepting), variant B (no accepting cycle; the loop runs until it
strips nothing, 1276 iterations).

Printed: one JSON line.  value = K * E / (step time) in GTEPS, K the number of
fixpoint computations and E the edge count: one traversal of every edge per
iteration, the least work any exact fixpoint needs.  The roofline object
prices the persistent loop kernel (the dominant kernel) at the method's bytes
per launch, K * (4E + 8N) (one pass over the column indices and row offsets
and one write of the map vector per fixpoint computation), over its average
launch time measured with HIP events on the launch stream; its `dense_equiv`
member prices the sweeps the schedule actually made as dense passes,
sweeps * (4(N+1) + 4E + 8N + N/8) + K * 4N, with sweeps counted over all
workgroups (their total over the number of workgroups).

The default line also carries `batched`: the first graphs of the config-4
batch solved in one persistent launch against the plain per-graph loop
(graphs/s, each verdict against the oracle's golden), and `cpu_baseline` with
its legs: the oracle's exact sequential route on one core (the headline
value), and the paper's propagation (jacobi) on one core and on all host
cores, on bounded samples of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MAP propagation GTEPS + HBM GB/s; graphs/s batched vs plain, bit-exact"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "c2B": ("config 2 variant B: N=2^20 state-space-shaped graph, no accepting cycle", "config2", False),
    "c2A": ("config 2 variant A: N=2^20 state-space-shaped graph, planted accepting 64-cycle", "config2", True),
    "c1a": ("config 1: N=10,000 uniform digraph, out-degree U{1..4}, 5% accepting", "config1", False),
    "c1b": ("config 1 DAG instance: high->low edges of the config-1 draw", "config1", True),
    "c3": ("config 3: N=2^25 DAG, ~134M edges, 0.1% accepting, no accepting cycle", "config3", None),
    "c3lit": ("config 3, literal reading: the config-1 generator at N=2^25 keeping edges with s > d (a DAG, "
              "~42M edges), 5% accepting, no accepting cycle", "config1lit", None),
    "c5": ("config 5: Poisson stream of config-1 DAG queries, N log-uniform in [1e4,4e6], accepting ratio "
           "U[0.1%,5%], odd ones planted; continuous batching on one persistent engine under a 32 GiB HBM budget "
           "vs a serial plain loop",
           "config5", None),
    "c4": ("config 4: 4,096 independent config-1 DAG graphs, N log-uniform in [1e3,1e6], odd ones with a "
           "planted accepting 64-cycle, one persistent launch vs the plain per-graph loop", "config4", None),
    "onthefly": ("detection on a growing graph: config 2 variant A's edge stream in generation order (grouped by "
                 "source), prefixes of 1/16, 2/16, ... each built, pruned (map_trim) and checked (map_detect) until "
                 "a cycle is found, vs one build + detection of the whole graph", "config2", True),
    "hub": ("hub rows: a config-3 style DAG with N=2^22 (~16.8M edges) plus four out-hubs of 10^5 edges, one "
            "graph solved by all workgroups through the batch path with the long-row threshold at its default "
            "(whole-wave fold) and off (every row folded by its own lane)", "config3", None),
    "lasso": ("counterexample on config 2 variant A: shortest path from vertex 1 to the witness found by "
              "map_detect, then shortest cycle through it (breadth-first search, one cooperative launch)",
              "config2", True),
}


def make_graph(key):
    import synth
    _, fn, flag = WORKLOADS[key]
    if fn == "config2":
        return synth.config2(planted=flag)
    if fn == "config1":
        return synth.config1(dag=flag)
    if fn == "config1lit":
        return synth.config1(seed=3, n=1 << 25, dag=True)
    return synth.config3()


def sweep_bytes(n, m):
    return 4 * (n + 1) + 4 * m + 8 * n + (n + 7) // 8


def method_bytes(n, m, k):
    """The method's minimum bytes for K fixpoint computations: per computation one
    pass over the CSR (4E column indices, 4N row offsets) and one write of map (4N)."""
    return k * (4 * m + 8 * n)


def host_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0))}


def golden_for(key):
    path = os.path.join(ROOT, "tests", "golden", "full_size.json")
    try:
        return json.load(open(path)).get(key)
    except (OSError, ValueError):
        return None


def _oracle_leg(g, mode, budget_s, omp=False, iters=None):
    """GTEPS_alg of the oracle's MAP loop on the first outer iterations that fit the budget."""
    import oracle
    if iters is None:
        probe = 1 if mode == "jacobi" else 5
        t = time.perf_counter()
        oracle.map_detect(g, mode=mode, max_iterations=probe, omp=omp)
        per = (time.perf_counter() - t) / probe
        iters = int(max(probe, min(10_000, budget_s / max(per, 1e-6))))
    t = time.perf_counter()
    d = oracle.map_detect(g, mode=mode, max_iterations=iters, omp=omp)
    dt = time.perf_counter() - t
    return d.iterations, dt, round(d.iterations * g.m / dt / 1e9, 6)


def cpu_baseline(g, key, budget_s=12.0, jacobi_budget_s=6.0):
    """The oracle (C, as it stands) on bounded samples: the exact sequential route
    on one core (the value), and the jacobi route on one core and on every
    host thread (the OpenMP build of the same source)."""
    import oracle
    k, dt, v = _oracle_leg(g, "desc", budget_s)
    out = {
        "value": v, "unit": "GTEPS", "cores": 1, "kind": "oracle",
        "sample": f"first {k} outer iterations of {key} (of the full run), oracle 'desc' fixpoint, "
                  f"{dt:.1f} s wall on the host",
        "host": host_info(),
    }
    kj, dtj, vj = _oracle_leg(g, "jacobi", jacobi_budget_s)
    kjo, dtjo, vjo = _oracle_leg(g, "jacobi", 0, omp=True, iters=kj)
    out["legs"] = [
        {"route": "desc", "cores": 1, "value": v, "unit": "GTEPS", "iterations": k, "seconds": round(dt, 3)},
        {"route": "jacobi", "cores": 1, "value": vj, "unit": "GTEPS", "iterations": kj, "seconds": round(dtj, 3)},
        {"route": "jacobi", "cores": oracle.threads(omp=True), "value": vjo, "unit": "GTEPS", "iterations": kjo,
         "seconds": round(dtjo, 3), "build": "OpenMP"},
    ]
    return out


def bench_batch(args):
    """Batched MAP over the config-4 graphs: graphs/s batched vs the plain loop."""
    figures = batch_run(args, args.batch_count)
    out = {
        "metric": METRIC, "value": figures.pop("graphs_per_s"), "unit": "graphs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": figures.pop("ms_per_step"),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": figures.pop("config"), **figures,
    }
    print(json.dumps(out), flush=True)


def batch_run(args, count, capture=True):
    """The first `count` config-4 graphs: one persistent launch (tuned gang policy)
    against the plain per-graph loop; returns the figures."""
    import torch
    import paper_0912_2555_amd as mc
    from paper_0912_2555_amd import autotune
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    csrs, accs, ns, ms, dmaxs = [], [], [], [], []
    ws = None
    for i in range(count):
        g = synth.config4(i)
        if ws is None or ws.numel() < mc.map_workspace_bytes(g.n, g.m):
            ws = mc.workspace(max(g.n, 1 << 20), max(g.m, 1 << 22), device=dev)
        # Both CSRs: the transposed one is read only by the direction-switch
        # option rules the tuner tries.
        csrs.append(mc.build_csr(g.n, g.src, g.dst, transposed=True, ws=ws))
        accs.append(torch.from_numpy(g.acc).to(dev))
        ns.append(g.n)
        ms.append(g.m)
        dmaxs.append(int(np.bincount(g.src).max()) if g.m else 0)
    torch.cuda.synchronize()
    print(f"[bench] c4: {count} graphs, sum n={sum(ns)} sum m={sum(ms)}, generated+uploaded in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    order = sorted(range(count), key=lambda i: -ms[i])       # largest first
    o_csrs = [csrs[i] for i in order]
    o_accs = [accs[i] for i in order]
    o_ns = [ns[i] for i in order]
    o_ms = [ms[i] for i in order]
    o_dmax = [dmaxs[i] for i in order]

    def make(gang, options=None):
        return mc.Batch(o_csrs, o_accs, gang=gang, device=dev, options=options)

    choice, timings = autotune.tune_knobs(make, o_ns, o_ms, o_dmax, torch.cuda.get_device_name(0), use_cache=False,
                                          log=lambda x: print(x, file=sys.stderr, flush=True))
    policy = choice["gang"]
    gang = autotune.gang_sizes(o_ns, o_ms, policy)
    options = autotune.graph_options(choice["options"], gang, o_ns, o_dmax)
    b = make(gang, options)
    for _ in range(args.warmup):
        b.launch()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        b.launch()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t) / args.steps
    res_b = b.read()

    # plain per-graph loop: one map_detect launch per graph, same order
    res_one = mc.new_result(dev)
    wsp = mc.workspace(max(ns), max(ms), device=dev)
    plain = []
    torch.cuda.synchronize()
    t = time.perf_counter()
    results_plain = torch.zeros((count, 8), dtype=torch.int32, device=dev)
    for j, c in enumerate(o_csrs):
        rc = mc.map_detect(c.n, c.row_ptr, c.col, None, None, o_accs[j], results_plain[j], None, None, 0,
                           mc.MAP_FLAG_NO_TRACE_DIGEST, wsp)
        if rc:
            raise mc.MapError(rc, "map_detect")
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t
    plain = [mc.Result.from_tensor(results_plain[j]) for j in range(count)]

    # the tuned launch captured in a HIP graph, replayed
    t_graph = None
    graph_ok = None
    bg = make(gang, options) if capture else None
    if bg is None:
        reps = 0
    else:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            bg.launch(stream=s)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        cg = torch.cuda.CUDAGraph()
        with torch.cuda.graph(cg):
            bg.launch()
        graph_ok = True
        reps = max(1, args.steps)
    for r in range(reps):
        bg.results.zero_()           # eager work between replays
        torch.cuda.synchronize()
        t = time.perf_counter()
        cg.replay()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        t_graph = dt if t_graph is None else min(t_graph, dt)
        graph_ok &= [x.verdict for x in bg.read()] == [x.verdict for x in res_b]

    exact_vs_plain = all(x.verdict == y.verdict and x.accepting_left == y.accepting_left and x.status == 0
                         and y.status == 0 for x, y in zip(res_b, plain))
    gold_path = os.path.join(ROOT, "tests", "golden", "batch_c4.json")
    exact_vs_oracle = None
    if os.path.exists(gold_path) and count <= 4096:
        gold = json.load(open(gold_path))["verdicts"]
        exact_vs_oracle = all([r.found, r.witness, r.iterations, r.accepting_left] == gold[i]
                              for r, i in zip(res_b, order))
    work = sum(r.iterations * m for r, m in zip(res_b, o_ms))
    return {
        "graphs_per_s": round(count / t_batch, 2), "ms_per_step": round(t_batch * 1e3, 3),
        "config": {"workload": WORKLOADS["c4"][0] if count == 4096 else
                   f"the first {count} of the 4,096 config-4 graphs", "key": "c4", "graphs": count,
                   "sum_n": int(sum(ns)),
                   "sum_m": int(sum(ms)), "parallelism": "single GPU", "order": "largest first",
                   "gang_policy": autotune.policy_name(policy), "option_rule": choice["options"]},
        "plain_graphs_per_s": round(count / t_plain, 2), "plain_ms": round(t_plain * 1e3, 3),
        "speedup_vs_plain": round(t_plain / t_batch, 3),
        "hipgraph_graphs_per_s": round(count / t_graph, 2) if t_graph else None,
        "hipgraph_replays_identical": graph_ok,
        "gteps_batch": round(work / t_batch / 1e9, 4),
        "tuner_ms": {k: round(v * 1e3, 3) for k, v in timings.items()},
        "exact_vs_plain": exact_vs_plain, "exact_vs_oracle_golden": exact_vs_oracle,
        "found": int(sum(r.found for r in res_b)),
    }


def hub_graph():
    """Config-3 generator at N=2^22 plus four out-hubs of 10^5 edges each."""
    import synth
    base = synth.config3(n=1 << 22)
    rng = np.random.default_rng(21)
    hubs = [np.stack([np.full(100_000, h, np.int64), rng.integers(1, h, 100_000)], 1)
            for h in ((1 << 22) - 3, 3 << 20, 1 << 21, 1 << 20)]
    e = np.concatenate([np.stack([base.src, base.dst], 1)] + hubs).astype(np.int32)
    return synth.Graph(n=base.n, src=e[:, 0].copy(), dst=e[:, 1].copy(), acc=base.acc, name="hub")


def bench_hub(args):
    """One hub graph through map_detect_batch with a gang of every workgroup:
    the long-row threshold at its default against off; both exact (oracle)."""
    import torch
    import oracle
    import paper_0912_2555_amd as mc
    torch.cuda.set_device(0)
    g = hub_graph()
    ref = oracle.map_detect(g, mode="desc")
    csr = mc.build_csr(g.n, g.src, g.dst, transposed=False)
    stream = torch.cuda.current_stream()
    out = {}
    for name, opt in (("whole_wave_fold", 0), ("lane_fold", mc.MAP_GRAPH_HUB_MASK)):
        b = mc.Batch([csr], [g.acc], gang=[1024], options=[opt])
        times = []
        for rep in range(args.warmup + args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            b.results.zero_()
            e0.record(stream)
            b.launch()
            e1.record(stream)
            torch.cuda.synchronize()
            if rep >= args.warmup:
                times.append(e0.elapsed_time(e1))
        r = b.read()[0]
        out[name] = {"ms": round(float(np.median(times)), 3), "exact": bool(r.verdict == ref.verdict and
                                                                             r.accepting_left == ref.accepting_left),
                     "sweeps": r.sweeps, "iterations": r.iterations}
    print(json.dumps({"workload": WORKLOADS["hub"][0], "n": g.n, "m": g.m, "hub_degree": 100_000, **out}),
          flush=True)


def bench_serve(args):
    """Serving: Poisson arrivals at rho x the serial plain throughput; p50/p99 and graphs/s.

    Query payloads (edge lists, flags) sit in pinned host memory, as a receive
    buffer would; the serial baseline and the server read the same buffers.
    """
    import torch
    import paper_0912_2555_amd as mc
    from paper_0912_2555_amd import autotune, serve
    import synth

    torch.cuda.set_device(0)
    count = args.serve_count
    t0 = time.perf_counter()
    graphs = [synth.config5(i) for i in range(count)]
    gaps = [synth.config5_meta(i)[2] for i in range(count)]
    pinned = [(torch.from_numpy(g.src).pin_memory(), torch.from_numpy(g.dst).pin_memory(),
               torch.from_numpy(g.acc).pin_memory()) for g in graphs]
    print(f"[bench] c5: {count} queries, sum n={sum(g.n for g in graphs)}, sum m={sum(g.m for g in graphs)}, "
          f"generated and pinned in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    def queries():
        return [serve.Query(i, g.n, p[0], p[1], p[2]) for i, (g, p) in enumerate(zip(graphs, pinned))]

    # serial plain throughput, saturated (back-to-back), on a sample
    sample = queries()[:min(count, 200)]
    serve.run_serial(sample[:4], qps=1e9)                      # warm-up
    sat, _ = serve.run_serial(sample, qps=1e9)
    rate = sat["graphs_per_s"]
    qps = args.rho * rate
    print(f"[bench] serial saturated {rate:.2f} graphs/s -> offered load {qps:.2f} queries/s", file=sys.stderr,
          flush=True)

    budget = 32 << 30
    # Engine mode (pull sweeps as map_detect, or filtered sweeps with the
    # direction switch) and gang policy: each candidate serves a sample of the
    # stream, all at once, on an engine of that mode.
    modes = {"pull": 0, "direction": mc.MAP_FLAG_DIRECTION}
    mode_names = list(modes) if args.serve_mode == "tune" else [args.serve_mode]
    tsample = queries()[:min(count, 200)]
    tuner, best = {}, None
    for mname in mode_names:
        with serve.Server(hbm_budget=budget, flags=modes[mname]) as srv:
            serve.run_stream(queries()[:16], qps=1e9, server=srv)  # warm-up

            def trial(pol):
                srv.gang_policy = (lambda ns, ms: autotune.gang_sizes(ns, ms, pol)) if pol else None
                return serve.run_stream([serve.Query(q.qid, q.n, q.src, q.dst, q.acc) for q in tsample],
                                        qps=1e9, server=srv)["span_s"]
            if args.serve_policy == "tune":
                pol, t = autotune.tune_by(trial, log=lambda x: print(f"[{mname}] {x}", file=sys.stderr, flush=True))
                tuner.update({f"{mname}|{k}": v for k, v in t.items()})
                span = t[autotune.policy_name(pol)]
            else:
                pol = autotune.parse_policy(args.serve_policy)
                span = trial(pol) if len(mode_names) > 1 else 0.0
                tuner[f"{mname}|{args.serve_policy}"] = span
        if best is None or span < best[0]:
            best = (span, mname, pol)
    _, mode, policy = best
    with serve.Server(hbm_budget=budget, flags=modes[mode]) as srv:
        warm = queries()[:16]
        serve.run_stream(warm, qps=1e9, server=srv)             # warm-up
        srv.gang_policy = (lambda ns, ms: autotune.gang_sizes(ns, ms, policy)) if policy else None
        srv.max_running = 0
        qs = queries()
        st = serve.run_stream(qs, qps=qps, server=srv, gaps=gaps)
        max_running = srv.max_running
        over = None
        if args.rho_over > 0:
            qo = queries()
            over = serve.run_stream(qo, qps=args.rho_over * rate, server=srv, gaps=gaps)
        qsat = queries()
        sat_engine = serve.run_stream(qsat, qps=1e9, server=srv)  # everything at once: engine capacity
        workgroups = srv.engine.workgroups
    ser, ser_res = serve.run_serial(queries(), qps=qps, gaps=gaps)
    exact = all(q.result.status == 0 and q.result.verdict == r.verdict and q.result.accepting_left == r.accepting_left
                for q, r in zip(qs, ser_res))
    exact_sat = all(a.result.verdict == b.result.verdict for a, b in zip(qsat, qs))
    rnd = lambda d: {k: round(v, 3) if isinstance(v, float) else v for k, v in d.items()}
    out = {
        "metric": METRIC, "value": round(st["graphs_per_s"], 3), "unit": "graphs/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": round(st["span_s"] * 1e3, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": WORKLOADS["c5"][0], "key": "c5", "queries": count, "rho": args.rho,
                   "offered_qps": round(qps, 3), "hbm_budget_gib": budget >> 30, "engine_workgroups": workgroups,
                   "gang_policy": autotune.policy_name(policy), "engine_mode": mode, "parallelism": "single GPU"},
        "serving": rnd(st),
        "serial_plain": rnd(ser),
        "serial_saturated_graphs_per_s": round(rate, 3),
        "engine_saturated": rnd(sat_engine),
        "overload": ({"rho": args.rho_over, **rnd(over)} if over else None),
        "max_queries_on_engine": max_running,
        "tuner_ms": ({k: round(v * 1e3, 2) for k, v in tuner.items()} if tuner else None),
        "exact_vs_serial": exact, "exact_saturated_vs_stream": exact_sat,
    }
    print(json.dumps(out), flush=True)


def bench_onthefly(args, chunks=16):
    """Growing-graph detection on the config-2A stream vs one detection of the whole graph."""
    import torch
    import paper_0912_2555_amd as mc
    from paper_0912_2555_amd import onthefly
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    g = synth.generation_order(make_graph("onthefly"))
    n, m = g.n, g.m
    print(f"[bench] onthefly on c2A stream n={n} m={m} chunks={chunks}", file=sys.stderr, flush=True)
    src = torch.from_numpy(g.src).to(dev)
    dst = torch.from_numpy(g.dst).to(dev)
    acc = torch.from_numpy(g.acc).to(dev)
    ws = mc.workspace(n, m, device=dev)
    for _ in range(args.warmup):
        onthefly.detect_stream(n, src, dst, acc, chunks=chunks, ws=ws)
    torch.cuda.synchronize()
    runs = []
    for _ in range(args.steps):
        runs.append(onthefly.detect_stream(n, src, dst, acc, chunks=chunks, ws=ws))
    torch.cuda.synchronize()
    best = min(runs, key=lambda r: r.total_ms)
    ms = float(np.median([r.total_ms for r in runs]))
    # the whole graph at once: pull CSR build + the MAP loop
    full = []
    for i in range(args.warmup + max(1, min(args.steps, 3))):
        t = time.perf_counter()
        csr = mc.build_csr(n, src, dst, transposed=False, ws=ws, device=dev)
        r = mc.detect(csr, acc, ws=ws).result
        if i >= args.warmup:
            full.append((time.perf_counter() - t) * 1e3)
    full_ms = float(np.median(full))
    pre = best.prefixes
    detect_ms = sum(p.detect_ms for p in pre)
    alg = sum(p.sweeps * sweep_bytes(n, p.edges) + p.iterations * 4 * n for p in pre)
    achieved = alg / (detect_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": round(ms, 3), "unit": "ms to verdict", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": WORKLOADS["onthefly"][0], "key": "onthefly", "n": n, "m": m, "chunks": chunks,
                   "parallelism": "single GPU"},
        "result": {"found": best.found, "witness": best.witness, "edges_at_verdict": best.edges_at_verdict,
                   "prefixes": [[p.edges, p.found, p.witness, p.iterations, p.kept, p.accepting_kept] for p in pre],
                   "stage_ms": {"build": round(sum(p.build_ms for p in pre), 3),
                                "trim": round(sum(p.trim_ms for p in pre), 3), "detect": round(detect_ms, 3)}},
        "whole_graph": {"ms": round(full_ms, 3), "found": r.found, "witness": r.witness, "iterations": r.iterations},
        "speedup_vs_whole_graph": round(full_ms / ms, 3),
        "roofline": {"bound": "hbm", "kernel": "map_loop_kernel", "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "bytes_per_launch": int(alg / max(len(pre), 1))},
    }
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        ref = []
        for c in range(1, chunks + 1):
            pm = m * c // chunks
            p = synth.prefix(g, pm)
            keep, pacc = oracle.trim(p)
            d = oracle.map_detect(p, pacc)
            ref.append([pm, d.found, d.witness, d.iterations, int(keep.sum()), int(pacc.sum())])
            if d.found:
                break
        cpu_s = time.perf_counter() - t
        out["result"]["matches_oracle"] = ref == out["result"]["prefixes"]
        out["cpu_baseline"] = {"value": round(cpu_s * 1e3, 1), "unit": "ms to verdict", "cores": 1,
                               "kind": "oracle", "sample": f"the same stream procedure on the oracle (trim + MAP per "
                                                           f"prefix, {len(ref)} prefixes), {cpu_s:.2f} s wall"}
    print(json.dumps(out), flush=True)


def bench_lasso(args):
    """Counterexample search on config 2A: map_detect gives the witness (untimed), then map_lasso is timed."""
    import torch
    import paper_0912_2555_amd as mc

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    g = make_graph("lasso")
    n, m = g.n, g.m
    print(f"[bench] lasso on c2A n={n} m={m}", file=sys.stderr, flush=True)
    csr = mc.build_csr(n, g.src, g.dst, transposed=False, device=dev)
    out = mc.detect(csr, g.acc)
    w = out.result.witness
    gold = golden_for("c2A")
    if out.result.found != 1 or (gold is not None and w != gold["witness"]):
        raise RuntimeError(f"map_detect gave found={out.result.found} witness={w}")
    init = 1
    ws = mc.workspace(n, m, device=dev)
    cap = 2 * n + 1
    path = torch.zeros(cap, dtype=torch.int32, device=dev)
    res = torch.zeros(8, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        rc = mc.map_lasso(n, csr.row_ptr, csr.col, w, init, path, res, ws)
        if rc:
            raise mc.MapError(rc, "map_lasso")
        if ev is not None:
            ev[1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(events[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    a = res.cpu().numpy()
    status, stem, cyc, plen = (int(x) for x in a[:4])
    scanned, levels = int(a[4:6].view(np.int64)[0]), int(a[6])
    if status != mc.MAP_OK:
        raise RuntimeError(f"map_lasso status {status}")
    import oracle
    t = time.perf_counter()
    ref = oracle.lasso(g, w, init)
    cpu_s = time.perf_counter() - t
    p = path[:plen].cpu().numpy().astype(np.int64)
    key = np.sort(g.src.astype(np.int64) * (n + 1) + g.dst)
    pk = p[:-1] * (n + 1) + p[1:]
    idx = np.minimum(np.searchsorted(key, pk), len(key) - 1)
    valid = bool(np.array_equal(key[idx], pk) and p[0] == init and p[stem] == w and p[-1] == w)
    ms_step = (t1 - t0) * 1e3 / args.steps
    lasso_ms = float(np.mean([x.elapsed_time(y) for x, y in events]))
    # two searches: each clears the n parent words; every examined edge reads its column and the
    # target's parent word
    alg_bytes = 2 * 4 * n + 8 * scanned
    achieved = alg_bytes / (lasso_ms * 1e-3) / 1e9
    result = {
        "metric": METRIC, "value": round(1e3 / ms_step, 2), "unit": "lassos/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": WORKLOADS["lasso"][0], "key": "lasso", "n": n, "m": m, "witness": w, "init": init,
                   "parallelism": "single GPU"},
        "result": {"stem_len": stem, "cycle_len": cyc, "path_len": plen, "edges_scanned": scanned,
                   "levels": levels, "path_valid": valid,
                   "lengths_match_oracle": bool((stem, cyc) == (ref.stem_len, ref.cycle_len))},
        "lasso_ms": round(lasso_ms, 4),
        "roofline": {"bound": "hbm", "kernel": "map_lasso_kernel", "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": None, "bytes_per_launch": int(alg_bytes)},
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = {"value": round(1.0 / cpu_s, 2), "unit": "lassos/s", "cores": 1, "kind": "oracle",
                                  "sample": f"one full lasso on c2A (stem from 1, cycle through {w}), "
                                            f"{cpu_s * 1e3:.1f} ms wall on the host"}
    print(json.dumps(result), flush=True)


def counted_traffic(workload: str, flags: int):
    """HBM bytes per launch from the committed counter summary, or None.

    The figure holds only for the workload and flags it was taken with and for
    the kernel source it was taken on; any other case reports None.
    """
    import hashlib
    import paper_0912_2555_amd as mc
    path = os.path.join(ROOT, "profiles", f"map_loop_kernel_{workload}_traffic.md")
    if not os.path.exists(path) or flags != mc.MAP_FLAG_NO_TRACE_DIGEST:
        return None
    kv = {}
    for line in open(path):
        key, sep, val = line.strip().partition(": ")
        if sep and key in ("source_sha256", "traffic_bytes_per_launch", "workload"):
            kv[key] = val.strip()
    src = os.path.join(ROOT, "paper_0912_2555_amd", "csrc", "mapcheck.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if kv.get("workload") != workload or kv.get("source_sha256") != digest:
        return None
    return int(kv["traffic_bytes_per_launch"])


def calibrate_copy(args):
    """A plain device copy of known size, for scaling the HBM traffic counters."""
    import torch
    nbytes = args.copy_mib << 20
    a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "device copy", "bytes_read": nbytes, "bytes_written": nbytes, "launches": 3}),
          flush=True)


PHASE_NAMES = ("setup", "remote_pass", "lds_passes", "stream_tiles", "report", "wait", "detect_strip", "other")


def phase_table(ph, iterations):
    """Per-phase breakdown of one loop-kernel launch from the measurement build's
    clocks (100 MHz ticks per workgroup): the mean over workgroups of each
    phase's time, its share, and the per-iteration and per-sweep figures."""
    ph = ph.astype(np.float64)
    nb = ph.shape[0]
    ms = ph[:, :8].mean(axis=0) / 1e5          # ticks of 10 ns -> ms
    total = float(ms.sum()) + float(ph[:, 12].mean() / 1e5) + float(ph[:, 13].mean() / 1e5)
    sweeps = ph[:, 8].mean()
    quiet = ph[:, 10].mean()
    lds = ph[:, 9].mean()
    table = {name: {"ms": round(float(v), 3), "share": round(float(v) / total, 4) if total else None}
             for name, v in zip(PHASE_NAMES, ms)}
    rw = float(ph[:, 12].mean() / 1e5)
    table["remote_pass_wait"] = {"ms": round(rw, 3), "share": round(rw / total, 4) if total else None}
    ga = float(ph[:, 13].mean() / 1e5)
    table["remote_gather"] = {"ms": round(ga, 3), "share": round(ga / total, 4) if total else None}
    return {
        "workgroups": nb, "launch_ms": round(total, 3), "per_phase": table,
        "per_workgroup_sweeps": round(float(sweeps), 1), "quiet_sweep_share": round(float(quiet / sweeps), 4)
        if sweeps else None,
        "lds_passes_per_sweep": round(float(lds / sweeps), 3) if sweeps else None,
        "us_per_iteration": round(total * 1e3 / iterations, 2) if iterations else None,
        "us_per_sweep": {"remote_pass": round(float(ms[1]) * 1e3 / sweeps, 3) if sweeps else None,
                         "lds_passes": round(float(ms[2]) * 1e3 / sweeps, 3) if sweeps else None},
        "us_per_lds_pass": round(float(ms[2]) * 1e3 / lds, 3) if lds else None,
    }


def single_run(args, workload, steps, warmup):
    """One graph: the CSR build and map_detect per step, timed as the main line
    describes; returns the line's fields and the graph (for the CPU leg)."""
    import torch
    import paper_0912_2555_amd as mc
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    g = make_graph(workload)
    n, m = g.n, g.m
    print(f"[bench] workload {workload} n={n} m={m} |A|={g.n_acc}", file=sys.stderr, flush=True)
    src = torch.from_numpy(g.src).to(dev)
    dst = torch.from_numpy(g.dst).to(dev)
    acc = torch.from_numpy(g.acc).to(dev)
    ws = mc.workspace(n, m, device=dev)
    row_ptr = torch.empty(n + 1, dtype=torch.int32, device=dev)
    col = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    # The transposed CSR is built only where the path reads it (frontier rounds,
    # the direction switch).
    # Config 3 (both readings) runs its filtered sweeps with the direction switch unless told not to.
    direction = not args.push and (args.direction or (workload in ("c3", "c3lit") and not args.pull_only))
    need_t = args.push or direction
    rrow_ptr = torch.empty(n + 1, dtype=torch.int32, device=dev) if need_t else None
    rcol = torch.empty(max(m, 1), dtype=torch.int32, device=dev) if need_t else None
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    res = mc.new_result(dev)
    stream = torch.cuda.current_stream()
    flags = mc.MAP_FLAG_NO_TRACE_DIGEST | (mc.MAP_FLAG_SYNC_SWEEPS if args.sync_sweeps else 0) | \
        (mc.MAP_FLAG_STREAM if args.stream else 0) | (mc.MAP_FLAG_PUSH if args.push else 0) | \
        (mc.MAP_FLAG_DIRECTION if direction else 0)

    def step(ev=None):
        rc = mc.map_build_csr(n, src, dst, row_ptr, col, rrow_ptr, rcol, status, ws)
        if rc:
            raise mc.MapError(rc, "map_build_csr")
        if ev is not None:
            ev[0].record(stream)
        rc = mc.map_detect(n, row_ptr, col, rrow_ptr, rcol, acc, res, None, None, 0, flags, ws)
        if rc:
            raise mc.MapError(rc, "map_detect")
        if ev is not None:
            ev[1].record(stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(events[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r = mc.Result.from_tensor(res)
    if r.status != 0 or int(status.item()) != 0:
        raise RuntimeError(f"device status {r.status} / build status {int(status.item())}")
    ms_step = (t1 - t0) * 1e3 / steps
    detect_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    k = r.iterations
    gteps = k * m / (ms_step * 1e-3) / 1e9
    alg_bytes = method_bytes(n, m, k)
    achieved = alg_bytes / (detect_ms * 1e-3) / 1e9
    dense_bytes = r.sweeps * sweep_bytes(n, m) + k * 4 * n
    dense_gbs = dense_bytes / (detect_ms * 1e-3) / 1e9
    traffic = counted_traffic(workload, flags)
    gold = golden_for(workload)
    exact = None
    if gold is not None:
        exact = bool((r.found, r.witness, r.iterations, r.accepting_left)
                     == (gold["found"], gold["witness"], gold["iterations"], gold["accepting_left"]))
    out = {
        "metric": METRIC, "value": round(gteps, 4), "unit": "GTEPS", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": WORKLOADS[workload][0], "key": workload, "n": n, "m": m,
                   "accepting": int(g.n_acc), "parallelism": "single GPU", "flags": flags},
        "result": {"found": r.found, "witness": r.witness, "iterations": k, "sweeps": r.sweeps,
                   "accepting_left": r.accepting_left, "matches_oracle_golden": exact},
        "detect_ms": round(detect_ms, 4), "build_ms": round(ms_step - detect_ms, 4),
        "gteps_detect": round(k * m / (detect_ms * 1e-3) / 1e9, 4),
        "gteps_scan": round(r.sweeps * m / (detect_ms * 1e-3) / 1e9, 4),
        "roofline": {"bound": "hbm", "kernel": "map_loop_kernel", "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "traffic_gbs": round(traffic / (detect_ms * 1e-3) / 1e9, 2) if traffic else None,
                     "bytes_per_launch": int(alg_bytes), "accounting": "method: K*(4E+8N) per launch",
                     "dense_equiv": {"achieved": round(dense_gbs, 2), "frac": round(dense_gbs / HBM_PEAK_GBS, 4),
                                     "bytes_per_launch": int(dense_bytes),
                                     "accounting": "whole-graph sweeps * (4(N+1)+4E+8N+N/8) + K*4N per launch"}},
    }
    return out, g, k


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2B", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--sync-sweeps", action="store_true", help="grid barrier after every sweep")
    ap.add_argument("--stream", action="store_true", help="stream the CSR every sweep (no on-chip staging)")
    ap.add_argument("--push", action="store_true", help="frontier rounds over the transposed CSR")
    ap.add_argument("--direction", action="store_true",
                    help="filtered sweeps switch to push rounds for small frontiers (builds the transposed CSR); "
                         "on by default for config 3")
    ap.add_argument("--pull-only", action="store_true", help="config 3 without the direction switch")
    ap.add_argument("--batch-count", type=int, default=4096, help="graphs in the config-4 batch")
    ap.add_argument("--line-c3", type=int, default=3,
                    help="timed config-3 steps added to the default config-2B line (0: none)")
    ap.add_argument("--line-batch", type=int, default=512,
                    help="single-graph line: also run the first N config-4 graphs batched vs plain (0: skip)")
    ap.add_argument("--phases", action="store_true",
                    help="load the phase-clock measurement build and add the per-phase breakdown of the last launch")
    ap.add_argument("--calibrate-copy", action="store_true", help="run a plain copy of known size and exit")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--serve-count", type=int, default=1000, help="queries in the config-5 stream")
    ap.add_argument("--rho", type=float, default=0.9, help="offered load / serial saturated throughput")
    ap.add_argument("--rho-over", type=float, default=1.5, help="second, overloaded stream (0: skip)")
    ap.add_argument("--serve-policy", default="tune",
                    help="gang policy when serving: tune, one, or EDGES[+fit] (edges per workgroup)")
    ap.add_argument("--serve-mode", default="tune", choices=["tune", "pull", "direction"],
                    help="engine sweeps when serving: pull (as map_detect) or filtered with the direction switch")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the detector runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding a graph by vertex range across GPUs is designed, not implemented)", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        calibrate_copy(args)
        return
    if args.workload == "c4":
        bench_batch(args)
        return
    if args.workload == "c5":
        bench_serve(args)
        return
    if args.workload == "lasso":
        bench_lasso(args)
        return
    if args.workload == "hub":
        bench_hub(args)
        return
    if args.workload == "onthefly":
        bench_onthefly(args)
        return

    if args.phases:
        os.environ["MAPCHECK_LIB"] = os.path.join(ROOT, "paper_0912_2555_amd", "libmapcheck_phases.so")
    import torch
    import paper_0912_2555_amd as mc

    out, g, k = single_run(args, args.workload, args.steps, args.warmup)
    if args.phases:
        out["phases"] = phase_table(mc.phase_counters(), k)
    if args.line_batch > 0:
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        out["batched"] = batch_run(args, args.line_batch, capture=False)
    if args.line_c3 > 0 and args.workload == "c2B" and not args.phases:
        # Config 3 (both CSRs built, filtered sweeps with the direction switch)
        # beside the headline config-2B figure.
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        c3, _, _ = single_run(args, "c3", args.line_c3, 1)
        out["config3"] = {key: c3[key] for key in ("value", "unit", "steps", "ms_per_step", "detect_ms", "build_ms",
                                                   "gteps_detect", "config", "result", "roofline")}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, args.workload, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
