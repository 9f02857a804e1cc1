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


def test_tune_knobs_retunes_the_gang_under_the_winning_rule(monkeypatch, tmp_path):
    """With a launch whose time depends on both knobs, the tuner takes the
    fastest gang policy at default options, the fastest rule on it, then the
    fastest gang policy under that rule -- here a different one -- and caches
    the pair."""
    import time
    import torch
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    monkeypatch.setenv("MAPCHECK_TUNE_CACHE", str(tmp_path / "tune.json"))
    ns, ms, dmax = [1000, 2000], [4000, 8000], [3, 4]
    one, wide = None, (1 << 14, False)
    fd = autotune.GRAPH_FILTER | autotune.GRAPH_DIRECTION
    # seconds per launch: default options favour `wide`; the direction rule is
    # faster still, and under it one workgroup per graph wins
    cost = {(autotune.policy_name(one), 0): 0.004, (autotune.policy_name(wide), 0): 0.002,
            (autotune.policy_name(one), fd): 0.0005, (autotune.policy_name(wide), fd): 0.001}

    class FakeBatch:
        def __init__(self, gangs, options):
            pol = one if gangs is None else wide
            opt = 0 if options is None else options[0]
            self.t = cost.get((autotune.policy_name(pol), opt), 0.003)

        def launch(self):
            time.sleep(self.t)

    choice, timings = autotune.tune_knobs(FakeBatch, ns, ms, dmax, "fake", reps=1, use_cache=True,
                                          gang_candidates=(one, wide),
                                          rules=("default", "filter-all", "direction-all"))
    assert choice == {"gang": one, "options": "direction-all"}, (choice, timings)
    assert "gang:one|direction-all" in timings
    assert "gang:16384|direction-all" not in timings        # the first stage's winner is not timed twice
    assert timings["gang:" + autotune.policy_name(wide)] < timings["gang:one"]
    again, _ = autotune.tune_knobs(FakeBatch, ns, ms, dmax, "fake", reps=1, use_cache=True,
                                   gang_candidates=(one, wide))
    assert again == choice                                  # from the cache
