"""Pins of the oracle's counterexample (lasso) search, CPU only.

The lasso for a witness w is a shortest path from an initial vertex to w and
a shortest cycle through w along edges of G (the paper lists counterexample
generation as missing from its tool, Section 5).  The oracle finds both by
breadth-first search; these pins fix it from outside:

* the hand example (tests/golden/hand_example.txt);
* closed forms: a relabelled simple cycle (the cycle is the only one), a chain
  leading into it (the stem is the chain), self-loops, DAGs (no cycle);
* brute force: shortest lengths from boolean matrix powers, an independent
  method, on random small digraphs, with every returned path checked edge by
  edge.  A reversed edge direction, an off-by-one level count or a stem that
  skips the witness fails one of them.
"""
import numpy as np
import pytest

import oracle
import synth
from conftest import read_golden


def _check_path(g, res, w, init):
    edges = set(zip(g.src.tolist(), g.dst.tolist()))
    p = res.path.tolist()
    assert len(p) == res.stem_len + res.cycle_len + 1
    assert p[0] == (init if init not in (0, w) else w)
    assert p[res.stem_len] == w and p[-1] == w
    for a, b in zip(p, p[1:]):
        assert (a, b) in edges, (a, b)


def test_hand_example():
    gold = read_golden("hand_example.txt")
    g = synth.from_edges(gold["n"][0][0], [tuple(e) for e in gold["edge"]], gold["accepting"][0])
    for w, init, s, c, *path in gold["lasso"]:
        r = oracle.lasso(g, w, init)
        assert (r.status, r.stem_len, r.cycle_len) == ("ok", s, c)
        assert r.path.tolist() == path
    for w, init in gold["lasso_none"]:
        assert oracle.lasso(g, w, init).status == "no_path"


@pytest.mark.parametrize("L", [1, 2, 3, 7, 40])
def test_relabelled_cycle_with_chain(L):
    rng = np.random.default_rng(L)
    chain = 5
    n = L + chain
    ids = rng.permutation(np.arange(1, n + 1))
    cyc, tail = ids[:L].tolist(), ids[L:].tolist()
    edges = [(cyc[i], cyc[(i + 1) % L]) for i in range(L)]
    edges += [(tail[i], tail[i + 1]) for i in range(chain - 1)] + [(tail[-1], cyc[0])]
    g = synth.from_edges(n, edges, [])
    for j, w in enumerate(cyc):
        r = oracle.lasso(g, w, 0)
        assert (r.status, r.cycle_len) == ("ok", L)
        assert r.path.tolist() == [cyc[(j + i) % L] for i in range(L)] + [w]
    r = oracle.lasso(g, cyc[0], tail[0])
    assert (r.status, r.stem_len, r.cycle_len) == ("ok", chain, L)
    assert r.path.tolist() == tail + cyc + [cyc[0]]
    # the chain vertices lie on no cycle, and the cycle cannot reach the chain
    assert oracle.lasso(g, tail[0], 0).status == "no_path"
    assert oracle.lasso(g, tail[0], cyc[0]).status == "no_path"


def test_self_loop_and_init_equal_to_witness():
    g = synth.from_edges(3, [(1, 2), (2, 2), (2, 3)], [2])
    r = oracle.lasso(g, 2, 1)
    assert (r.status, r.stem_len, r.cycle_len, r.path.tolist()) == ("ok", 1, 1, [1, 2, 2])
    r = oracle.lasso(g, 2, 2)
    assert (r.stem_len, r.cycle_len, r.path.tolist()) == (0, 1, [2, 2])


def test_dag_has_no_cycle():
    g = synth.config1(seed=1, n=200, dag=True)
    for w in range(1, 201, 17):
        assert oracle.lasso(g, w, 0).status == "no_path"


def test_capacity():
    g = synth.from_edges(3, [(1, 2), (2, 3), (3, 1)], [])
    assert oracle.lasso(g, 1, 0, cap=3).status == "no_space"
    r = oracle.lasso(g, 1, 0, cap=4)
    assert r.status == "ok" and r.path.tolist() == [1, 2, 3, 1]


def _powers(g, n):
    """dist[k][u][v]: u reaches v by a walk of exactly k edges, k = 0..n."""
    a = np.zeros((n, n), bool)
    a[g.src - 1, g.dst - 1] = True
    p = [np.eye(n, dtype=bool)]
    for _ in range(n):
        p.append((p[-1].astype(np.int32) @ a.astype(np.int32)) > 0)
    return p


@pytest.mark.parametrize("seed", range(40))
def test_brute_force_lengths(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(2, 11))
    m = int(rng.integers(1, 3 * n))
    edges = [(int(rng.integers(1, n + 1)), int(rng.integers(1, n + 1))) for _ in range(m)]
    g = synth.from_edges(n, edges, [])
    p = _powers(g, n)
    for w in range(1, n + 1):
        cyc = next((k for k in range(1, n + 1) if p[k][w - 1, w - 1]), -1)
        for init in range(0, n + 1):
            r = oracle.lasso(g, w, init)
            stem = 0 if init in (0, w) else next((k for k in range(1, n) if p[k][init - 1, w - 1]), -1)
            if stem < 0 or cyc < 0:
                assert r.status == "no_path"
                continue
            assert (r.status, r.stem_len, r.cycle_len) == ("ok", stem, cyc)
            _check_path(g, r, w, init)


def _all_walks(adj, a, b, k):
    """Every walk of exactly k edges from a to b (k >= 1), as vertex lists."""
    out = []

    def go(path):
        if len(path) == k + 1:
            if path[-1] == b:
                out.append(list(path))
            return
        for v in adj[path[-1]]:
            path.append(v)
            go(path)
            path.pop()

    go([a])
    return out


def _canonical(walks):
    """Of several shortest walks, the one whose vertices read backwards are
    lexicographically smallest."""
    return min(walks, key=lambda p: p[::-1])


@pytest.mark.parametrize("seed", range(40))
def test_brute_force_canonical_paths(seed):
    """Dense small digraphs with many shortest paths: every shortest walk is
    enumerated and the backwards-smallest one must be the oracle's stem and
    cycle (the choice depends on the edge set only, so a shuffled edge list
    gives the same path)."""
    rng = np.random.default_rng(2000 + seed)
    n = int(rng.integers(3, 8))
    m = int(rng.integers(n, 4 * n))
    edges = [(int(rng.integers(1, n + 1)), int(rng.integers(1, n + 1))) for _ in range(m)]
    g = synth.from_edges(n, edges, [])
    shuffled = synth.from_edges(n, [edges[i] for i in rng.permutation(m)], [])
    adj = {u: sorted({b for a, b in edges if a == u}) for u in range(1, n + 1)}
    several = 0
    for w in range(1, n + 1):
        r = oracle.lasso(g, w, 0)
        if r.status != "ok":
            continue
        walks = _all_walks(adj, w, w, r.cycle_len)
        several += len(walks) > 1
        assert r.path.tolist() == _canonical(walks)
        for init in range(1, n + 1):
            if init == w:
                continue
            r = oracle.lasso(g, w, init)
            if r.status != "ok":
                continue
            stem = _canonical(_all_walks(adj, init, w, r.stem_len))
            cyc = _canonical(_all_walks(adj, w, w, r.cycle_len))
            assert r.path.tolist() == stem + cyc[1:], (init, w)
            assert oracle.lasso(shuffled, w, init).path.tolist() == r.path.tolist()
    if seed == 0:
        assert several > 0
