"""Batched MAP captured in a HIP graph and tuned by the autotuner, through the
C ABI: every replay of a captured launch -- one workgroup per graph (an
ordinary launch) and gangs of workgroups (a cooperative launch) -- gives every
graph the oracle's result, with the program's own eager work and
synchronizations between the replays; the autotuner's choice of both knobs
(gang policy, per-graph options) gives the oracle's results too."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    import paper_0912_2555_amd as mc
    return mc


@pytest.fixture(scope="module")
def batch():
    gs = [synth.config4(i) for i in range(20)]
    gs.append(synth.config2(seed=12, n=1 << 15, planted=True))
    refs = [oracle.map_detect(g, mode="desc") for g in gs]
    order = sorted(range(len(gs)), key=lambda i: -gs[i].m)
    return [gs[i] for i in order], [refs[i] for i in order]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _exact(res, refs):
    return all(r.status == 0 and r.verdict == f.verdict and r.accepting_left == f.accepting_left
               for r, f in zip(res, refs))


@pytest.mark.parametrize("policy", ["one-per-graph", "gangs", "one-per-graph-direction", "gangs-direction"])
def test_captured_batch_replays_exact(mc, batch, policy):
    import torch
    gs, refs = batch
    direction = policy.endswith("-direction")
    csrs = [mc.build_csr(g.n, g.src, g.dst, transposed=direction) for g in gs]
    gang = None if policy.startswith("one-per-graph") else [1 if g.n < 20_000 else 4 for g in gs]
    if direction:   # filtered sweeps with the direction switch on most graphs, plain ones between
        options = [0 if i % 4 == 3 else mc.MAP_GRAPH_FILTER | mc.MAP_GRAPH_DIRECTION for i in range(len(gs))]
    else:
        options = [mc.MAP_GRAPH_SYNC_SWEEPS if i % 3 == 0 else 0 for i in range(len(gs))]
    b = mc.Batch(csrs, [g.acc for g in gs], gang=gang, options=options)
    say("capture", policy, "graphs", len(gs))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.launch(stream=s)           # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    assert _exact(b.read(), refs)
    cg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(cg):
        b.launch()
    for rep in range(3):
        b.results.zero_()            # eager work between the replays
        scratch = torch.arange(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        cg.replay()
        torch.cuda.synchronize()
        assert int(scratch) == (1 << 16) * ((1 << 16) - 1) // 2
        res = b.read()
        say("  replay", rep, "found", sum(r.found for r in res))
        assert _exact(res, refs), rep


def test_tuned_knobs_exact(mc, batch):
    import torch
    from paper_0912_2555_amd import autotune
    gs, refs = batch
    # Both CSRs, so that the direction-switch rules the tuner tries take effect.
    csrs = [mc.build_csr(g.n, g.src, g.dst, transposed=True) for g in gs]
    ns, ms = [g.n for g in gs], [g.m for g in gs]
    dmax = [int(np.bincount(g.src).max()) if g.m else 0 for g in gs]

    def make(gang, options=None):
        return mc.Batch(csrs, [g.acc for g in gs], gang=gang, options=options)

    choice, timings = autotune.tune_knobs(make, ns, ms, dmax, torch.cuda.get_device_name(0), reps=1,
                                          use_cache=False,
                                          gang_candidates=(None, (1 << 15, False), (1 << 14, True)))
    say("tuned", choice, {k: round(v * 1e3, 2) for k, v in timings.items()})
    assert choice["options"] in autotune.OPTION_RULES
    assert any(k.startswith("options:") for k in timings) and any(k.startswith("gang:") for k in timings)
    gang = autotune.gang_sizes(ns, ms, choice["gang"])
    b = make(gang, autotune.graph_options(choice["options"], gang, ns, dmax))
    b.launch()
    torch.cuda.synchronize()
    assert _exact(b.read(), refs)
