"""Batched MAP (many graphs, one persistent launch): every graph's result is
identical to the oracle's and to the single-graph call (bit-exact)."""
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


def _mixed_graphs():
    gs = [synth.config4(i) for i in range(0, 12)]                  # c4 members (1e3..1e6 vertices)
    gs += [synth.random_graph(500 + i, n, int(n * 1.5), p_acc=0.1) for i, n in enumerate([1, 2, 64, 129, 3000])]
    gs += [synth.config1(seed=8), synth.config1(seed=8, dag=True), synth.config2(seed=9, n=1 << 14, planted=True)]
    gs += [synth.from_edges(5, [(1, 2), (2, 3), (3, 1), (3, 4), (4, 5)], [2, 4, 5], "hand"),
           synth.from_edges(3, [], [], "empty-acc")]
    return gs


@pytest.fixture(scope="module")
def graphs():
    gs = _mixed_graphs()
    refs = [oracle.map_detect(g, mode="desc") for g in gs]
    return gs, refs


def _check(mc, gs, refs, gang=None, flags=0, order=None, options=None, transposed=False):
    order = list(range(len(gs))) if order is None else order
    csrs = [mc.build_csr(gs[i].n, gs[i].src, gs[i].dst, transposed=transposed) for i in order]
    opts = None if options is None else [options[i] for i in order]
    b = mc.Batch(csrs, [gs[i].acc for i in order], gang=gang, flags=flags, options=opts)
    b.launch()
    res = b.read()
    for r, i in zip(res, order):
        ref = refs[i]
        assert r.status == 0, (gs[i].name, r)
        assert r.verdict == ref.verdict, (gs[i].name, r.verdict, ref.verdict)
        assert r.accepting_left == ref.accepting_left, gs[i].name
    return res


def test_batch_one_block_per_graph(mc, graphs):
    gs, refs = graphs
    _check(mc, gs, refs)


def test_batch_largest_first_and_repeat(mc, graphs):
    gs, refs = graphs
    order = sorted(range(len(gs)), key=lambda i: -gs[i].m)
    a = _check(mc, gs, refs, order=order)
    b = _check(mc, gs, refs, order=order)
    assert [x.verdict for x in a] == [x.verdict for x in b]


@pytest.mark.parametrize("policy", ["gang4", "mixed", "wide"])
def test_batch_gangs(mc, graphs, policy):
    gs, refs = graphs
    if policy == "gang4":
        gang = [4] * len(gs)
    elif policy == "mixed":
        gang = [1 if g.n < 20000 else min(16, 1 + g.n // 20000) for g in gs]
    else:  # gangs beyond 64 workgroups, up to more than the grid holds (clamped by the library)
        gang = [[96, 200, 1000][i % 3] for i in range(len(gs))]
    _check(mc, gs, refs, gang=gang)


@pytest.mark.parametrize("flags", ["stream", "sync"])
def test_batch_modes(mc, graphs, flags):
    gs, refs = graphs
    f = mc.MAP_FLAG_STREAM if flags == "stream" else mc.MAP_FLAG_SYNC_SWEEPS
    _check(mc, gs, refs, gang=[2] * len(gs), flags=f)


def test_batch_matches_single_graph_calls(mc, graphs):
    gs, refs = graphs
    res = _check(mc, gs, refs)
    for g, r in zip(gs, res):
        csr = mc.build_csr(g.n, g.src, g.dst, transposed=False)
        single = mc.detect(csr, g.acc).result
        assert single.verdict == r.verdict and single.accepting_left == r.accepting_left


def test_batch_workspace_too_small_reports(mc, graphs):
    import torch
    gs, refs = graphs
    csrs = [mc.build_csr(g.n, g.src, g.dst, transposed=False) for g in gs[:3]]
    b = mc.Batch(csrs, [g.acc for g in gs[:3]])
    b.total_n = 3  # understate the size: the device check must refuse
    b.ws = torch.empty(mc.map_batch_workspace_bytes(3, 3), dtype=torch.uint8, device="cuda")
    b.launch()
    assert all(r.status == mc.MAP_ENOSPC for r in b.read())


def _hub_graph():
    """Out-hubs of 20,000 edges (many staged chunks) on a config-1 base."""
    base = synth.config1(seed=11, n=50_000)
    rng = np.random.default_rng(11)
    hubs = [np.stack([np.full(20_000, h), rng.integers(1, base.n + 1, 20_000)], 1) for h in (5, 25_000)]
    e = np.concatenate([np.stack([base.src, base.dst], 1)] + hubs).astype(np.int32)
    return synth.Graph(n=base.n, src=e[:, 0].copy(), dst=e[:, 1].copy(), acc=base.acc, name="c1-hubs")


@pytest.mark.parametrize("opt", ["hub1", "hub8", "hub-never", "sync", "stream", "stream+sync+hub16", "filter",
                                 "filter+hub8", "direction"])
def test_batch_per_graph_options(mc, graphs, opt):
    """Per-graph options (long-row threshold, barrier per sweep, streamed CSR,
    filtered sweeps) on every other graph, the hub graph among them: every
    result exact."""
    gs, refs = graphs
    gs = gs + [_hub_graph()]
    refs = refs + [oracle.map_detect(gs[-1], mode="desc")]
    o = {"hub1": 1, "hub8": 8, "hub-never": mc.MAP_GRAPH_HUB_MASK, "sync": mc.MAP_GRAPH_SYNC_SWEEPS,
         "stream": mc.MAP_GRAPH_STREAM,
         "stream+sync+hub16": mc.MAP_GRAPH_STREAM | mc.MAP_GRAPH_SYNC_SWEEPS | 16,
         "filter": mc.MAP_GRAPH_FILTER, "filter+hub8": mc.MAP_GRAPH_FILTER | 8,
         "direction": mc.MAP_GRAPH_FILTER | mc.MAP_GRAPH_DIRECTION}[opt]
    options = [o if i % 2 == 0 or i == len(gs) - 1 else 0 for i in range(len(gs))]
    _check(mc, gs, refs, gang=[1 if g.n < 20000 else 4 for g in gs], options=options,
           transposed=opt == "direction")
