"""Pins of the oracle's relevance pruning (trim of cycle-free vertices), CPU only.

The trim repeatedly removes a vertex with no remaining predecessor or no
remaining successor; what remains is the largest set in which every vertex has
a predecessor and a successor inside the set.  It stands in, on a bare graph,
for the paper's reduction to components that contain accepting states
(Section 2).  Pins:

* a hand case with two cycles, the path between them and a source tail;
* an independent method: the greatest fixpoint S = {v in S : some edge u->v
  and some edge v->w with u, w in S}, iterated from S = all vertices with
  vectorised numpy, on random graphs of several densities;
* every vertex of a nontrivial strongly connected component or on a self-loop
  (Tarjan) is kept, and the kept set is closed as defined;
* DAGs trim to nothing;
* the verdict with the pruned accepting set equals the verdict without
  pruning, exhaustively on every graph with n <= 3 and every accepting set,
  and on random graphs.
"""
import numpy as np
import pytest

import oracle
import synth


def _g(n, edges, acc):
    return synth.from_edges(n, edges, acc)


def test_hand_case():
    # cycle 1-2-3, path 3->4->5, cycle 5-6, source tail 7->1, sink tail 6->8->9
    g = _g(9, [(1, 2), (2, 3), (3, 1), (3, 4), (4, 5), (5, 6), (6, 5), (7, 1), (6, 8), (8, 9)], [1, 4, 7, 9])
    keep, acc = oracle.trim(g)
    assert keep.tolist() == [1, 1, 1, 1, 1, 1, 0, 0, 0]
    assert acc.tolist() == [1, 0, 0, 1, 0, 0, 0, 0, 0]


def _naive(g):
    s = np.ones(g.n, bool)
    src, dst = g.src - 1, g.dst - 1
    while True:
        has_in = np.zeros(g.n, bool)
        has_out = np.zeros(g.n, bool)
        live = s[src] & s[dst]
        has_in[dst[live]] = True
        has_out[src[live]] = True
        t = s & has_in & has_out
        if np.array_equal(t, s):
            return s
        s = t


def _random(seed, n, deg):
    rng = np.random.default_rng(seed)
    m = int(n * deg)
    src = rng.integers(1, n + 1, m).astype(np.int32)
    dst = rng.integers(1, n + 1, m).astype(np.int32)
    acc = (rng.random(n) < 0.2).astype(np.uint8)
    return synth.Graph(n=n, src=src, dst=dst, acc=acc, name=f"r{seed}")


@pytest.mark.parametrize("seed,n,deg", [(s, n, d) for s, (n, d) in enumerate(
    [(5, 0.5), (30, 0.8), (30, 1.0), (200, 0.9), (200, 1.1), (1000, 1.0), (1000, 1.5), (5000, 0.7), (5000, 1.0),
     (20000, 1.2)])])
def test_equals_naive_fixpoint_and_contains_cycles(seed, n, deg):
    g = _random(seed, n, deg)
    keep, acc = oracle.trim(g)
    assert np.array_equal(keep.astype(bool), _naive(g))
    assert np.array_equal(acc, g.acc & keep)
    # closed: every kept vertex has a kept predecessor and a kept successor
    k = keep.astype(bool)
    live = k[g.src - 1] & k[g.dst - 1]
    assert set(np.nonzero(k)[0].tolist()) <= set((g.dst[live] - 1).tolist())
    assert set(np.nonzero(k)[0].tolist()) <= set((g.src[live] - 1).tolist())
    # every vertex of a nontrivial SCC, or on a self-loop, is kept
    if n <= 5000:
        _, comp = oracle.tarjan(g, with_components=True)
        sizes = np.bincount(comp)
        on_cycle = sizes[comp] >= 2
        on_cycle[g.src[g.src == g.dst] - 1] = True
        assert np.all(k[on_cycle])


def test_dags_trim_to_nothing():
    for g in (synth.config1(dag=True), synth.config3(n=1 << 12)):
        keep, acc = oracle.trim(g)
        assert keep.sum() == 0 and acc.sum() == 0


def _all_graphs(n):
    pairs = [(s, d) for s in range(1, n + 1) for d in range(1, n + 1)]
    for mask in range(1 << len(pairs)):
        edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        for amask in range(1 << n):
            yield edges, [v for v in range(1, n + 1) if amask >> (v - 1) & 1]


def test_verdict_preserved_exhaustive_n_le_3():
    for n in (1, 2, 3):
        for edges, acc in _all_graphs(n):
            g = _g(n, edges, acc)
            keep, pacc = oracle.trim(g)
            assert np.array_equal(keep.astype(bool), _naive(g)), (n, edges)
            assert oracle.map_detect(g, pacc).found == oracle.map_detect(g).found == oracle.tarjan(g), (n, edges, acc)


@pytest.mark.parametrize("seed", range(20))
def test_verdict_preserved_random(seed):
    g = _random(100 + seed, 400, 0.6 + 0.05 * seed)
    keep, pacc = oracle.trim(g)
    full = oracle.map_detect(g)
    pruned = oracle.map_detect(g, pacc)
    assert pruned.found == full.found == oracle.tarjan(g)
    if full.found:
        assert pruned.witness > 0 and keep[pruned.witness - 1] == 1
