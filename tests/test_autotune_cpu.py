"""Host logic of the batch autotuner (CPU only): gang sizes of a policy and the
per-graph options each option rule gives a graph class."""
from paper_0912_2555_amd import autotune


def test_gang_sizes_and_names():
    ns, ms = [10, 5000, 2_000_000], [20, 20_000, 5_000_000]
    assert autotune.gang_sizes(ns, ms, None) is None
    assert autotune.gang_sizes(ns, ms, (1 << 14, False)) == [1, 2, 256]
    assert autotune.gang_sizes(ns, ms, (1 << 20, True)) == [1, 2, 256]  # raised to fit n, then capped
    assert autotune.gang_sizes([600_000], [100_000], (1 << 20, False)) == [1]
    assert autotune.gang_sizes([600_000], [100_000], (1 << 20, True)) == [147]  # ceil(600000 / 4096)
    for p in autotune.CANDIDATES:
        assert autotune.parse_policy(autotune.policy_name(p)) == p


def test_option_rules():
    gangs, ns, dmax = [1, 2, 16], [100, 50_000, 900_000], [3, 40, 100_000]
    o = lambda rule: autotune.graph_options(rule, gangs, ns, dmax)
    assert o("default") == [0, 0, 0]
    assert o("sync-gangs") == [0, autotune.GRAPH_SYNC_SWEEPS, autotune.GRAPH_SYNC_SWEEPS]
    assert o("sync-small-gangs") == [0, autotune.GRAPH_SYNC_SWEEPS, 0]
    assert o("stream-single") == [autotune.GRAPH_STREAM, 0, 0]
    assert o("hub8") == [0, 8, 8]
    assert o("hub-never") == [autotune.HUB_NEVER] * 3
    assert o("filter-gangs") == [0, autotune.GRAPH_FILTER, autotune.GRAPH_FILTER]
    assert o("filter-all") == [autotune.GRAPH_FILTER] * 3
    fd = autotune.GRAPH_FILTER | autotune.GRAPH_DIRECTION
    assert o("direction-gangs") == [0, fd, fd]
    assert o("direction-all") == [fd] * 3
    # gangs None: one workgroup per graph
    assert autotune.graph_options("stream-single", None, ns, dmax) == [autotune.GRAPH_STREAM] * 3


def test_option_bits_match_the_header():
    import os
    import re
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    text = open(os.path.join(root, "include", "mapcheck.h")).read()
    vals = dict(re.findall(r"#define (MAP_GRAPH_\w+) (0x[0-9a-fA-F]+)", text))
    assert int(vals["MAP_GRAPH_SYNC_SWEEPS"], 16) == autotune.GRAPH_SYNC_SWEEPS
    assert int(vals["MAP_GRAPH_STREAM"], 16) == autotune.GRAPH_STREAM
    assert int(vals["MAP_GRAPH_HUB_MASK"], 16) == autotune.HUB_NEVER
    assert int(vals["MAP_GRAPH_FILTER"], 16) == autotune.GRAPH_FILTER
    assert int(vals["MAP_GRAPH_DIRECTION"], 16) == autotune.GRAPH_DIRECTION
