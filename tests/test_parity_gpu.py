"""Parity of the HIP library (through its C ABI) with the CPU oracle.

Integer work: every comparison is bit-exact -- found flag, witness, K, the
accepting set at exit, per-iteration |Del_k| and map digests, and full map
vectors where the oracle can produce them.  Sweep counts depend on the
schedule and are not compared.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def mc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    import paper_0912_2555_amd as mc
    return mc


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def accepting_sequence(g, ref):
    """A_1..A_K reconstructed from the oracle's map vectors."""
    acc = g.acc.copy()
    out = []
    for k in range(min(ref.iterations, len(ref.maps))):
        out.append(acc.copy())
        nz = ref.maps[k][ref.maps[k] != 0]
        acc[nz - 1] = 0
    return out


def check_detect(mc, g, csr=None, max_iterations=0, trace_cap=None, flags=0, ref=None):
    say("detect", g.name, "n", g.n, "m", g.m)
    if csr is None:
        csr = mc.build_csr(g.n, g.src, g.dst)
    if ref is None:
        ref = oracle.map_detect(g, mode="desc", max_iterations=max_iterations)
    cap = (g.n_acc + 1) if trace_cap is None else trace_cap
    out = mc.detect(csr, g.acc, trace_cap=cap, want_acc=True, max_iterations=max_iterations, flags=flags)
    r = out.result
    want_status = 0 if ref.status == 0 else mc.MAP_ENOTCONVERGED
    assert r.status == want_status, (g.name, r)
    assert r.verdict == ref.verdict, (g.name, r, ref.verdict)
    assert r.accepting_left == ref.accepting_left
    assert np.array_equal(out.accepting_out, ref.acc_out)
    rows = min(r.iterations, cap)
    assert out.trace.shape[0] == rows
    assert np.array_equal(out.trace[:, 0], ref.trace[:rows, 0].astype(np.uint64)), g.name
    if not flags & mc.MAP_FLAG_NO_TRACE_DIGEST:
        assert np.array_equal(out.trace[:, 2], ref.trace[:rows, 2].astype(np.uint64)), g.name
    assert np.all(out.trace[:, 1] >= 1)
    assert r.sweeps == int(out.trace[:, 1].sum()) or rows < r.iterations
    return out, ref


def check_propagate_all(mc, g, csr=None, max_k=None, flags=0):
    """Full map vector of every iteration (the oracle's A_k as input)."""
    if csr is None:
        csr = mc.build_csr(g.n, g.src, g.dst)
    ref = oracle.map_detect(g, mode="jacobi" if g.n <= 20000 else "desc", maps_cap=max_k or (g.n_acc + 1))
    accs = accepting_sequence(g, ref)
    for k, acc in enumerate(accs[:max_k]):
        got, res = mc.propagate(csr, acc, flags=flags)
        assert res.status == 0
        assert np.array_equal(got.cpu().numpy(), ref.maps[k]), (g.name, k + 1)
    return ref


# ------------------------------------------------------------------ small

def test_hand_example(mc):
    from conftest import read_golden
    gold = read_golden("hand_example.txt")
    g = synth.from_edges(gold["n"][0][0], [tuple(e) for e in gold["edge"]], gold["accepting"][0], "hand")
    out, _ = check_detect(mc, g)
    assert list(out.result.verdict) == gold["result"][0]
    check_propagate_all(mc, g)


@pytest.mark.parametrize("dag", [False, True], ids=["c1a", "c1b"])
def test_config1_full_vectors(mc, dag):
    g = synth.config1(dag=dag)
    csr = mc.build_csr(g.n, g.src, g.dst)
    check_detect(mc, g, csr)
    check_propagate_all(mc, g, csr)


def _random_cases():
    cases = []
    for i, (n, deg) in enumerate([(1, 1), (2, 2), (3, 3), (63, 2), (64, 3), (65, 1), (127, 4), (128, 2),
                                  (129, 3), (1000, 1.2), (1000, 3), (4099, 2), (20000, 1.1), (40000, 2.5),
                                  (70001, 1.5)]):
        m = max(0, int(n * deg))
        cases.append(synth.random_graph(100 + i, n, m, p_acc=0.05 if n > 100 else 0.3))
    return cases


@pytest.mark.parametrize("g", _random_cases(), ids=lambda g: g.name)
def test_random_graphs(mc, g):
    csr = mc.build_csr(g.n, g.src, g.dst)
    check_detect(mc, g, csr)
    check_propagate_all(mc, g, csr, max_k=4)


@pytest.mark.parametrize("g", [c for c in _random_cases() if c.n >= 64] + [synth.config1(dag=True),
                               synth.config2(seed=3, n=1 << 15, planted=True),
                               synth.config2(seed=6, n=1 << 14)], ids=lambda g: g.name)
@pytest.mark.parametrize("filt", [True, False], ids=["filtered", "unfiltered"])
def test_stream_mode(mc, g, filt):
    """The same results with the CSR streamed every sweep instead of staged on
    chip: by default with a barrier per sweep and gathers only from rows that
    grew in the previous sweep, and with that filter off (asynchronous)."""
    flags = mc.MAP_FLAG_STREAM | (0 if filt else mc.MAP_FLAG_NO_FILTER)
    csr = mc.build_csr(g.n, g.src, g.dst)
    check_detect(mc, g, csr, flags=flags)
    ref = oracle.map_detect(g, mode="desc", maps_cap=1)
    got, res = mc.propagate(csr, g.acc, flags=flags)
    assert res.status == 0 and np.array_equal(got.cpu().numpy(), ref.maps[0])


@pytest.mark.parametrize("g", [synth.config3(n=1 << 16), synth.config2(seed=8, n=1 << 13, planted=True),
                               synth.config1()], ids=lambda g: g.name)
def test_filtered_stream_full_vectors(mc, g):
    """Filtered stream sweeps (barrier per sweep, gathers only from rows that
    grew): the full map vector of every iteration equals the oracle's."""
    check_propagate_all(mc, g, max_k=8, flags=mc.MAP_FLAG_STREAM)


def _chain_graph(n, acc_every):
    """v -> v+1 for every v, accepting every acc_every-th vertex: each sweep
    grows a handful of rows (push rounds throughout the direction switch)."""
    edges = [(v, v + 1) for v in range(1, n)] + [(n, 1)] * (n % 7 == 0)
    return synth.from_edges(n, edges, range(acc_every, n + 1, acc_every), f"chain{n}")


@pytest.mark.parametrize("g", [synth.config3(n=1 << 16), synth.config2(seed=8, n=1 << 13, planted=True),
                               synth.config2(seed=9, n=1 << 15), synth.config1(), synth.config1(dag=True),
                               _chain_graph(3000, 250), _chain_graph(2800, 97)], ids=lambda g: g.name)
def test_direction_switch_full_vectors(mc, g):
    """Filtered stream sweeps with the direction switch (push rounds from the
    rows that grew while they are fewer than n/16, pull sweeps otherwise):
    every iteration's full map vector and the whole detection equal the
    oracle's."""
    flags = mc.MAP_FLAG_STREAM | mc.MAP_FLAG_DIRECTION
    csr = mc.build_csr(g.n, g.src, g.dst)
    check_propagate_all(mc, g, csr, max_k=6, flags=flags)
    check_detect(mc, g, csr, flags=flags)


def test_direction_switch_dense_and_hubs(mc):
    """Dense random digraphs (frontiers large enough for pull sweeps between
    push rounds) and the hub graph (a push from a row with 50,000
    predecessors)."""
    rng = np.random.default_rng(41)
    for n, deg in ((5000, 8), (40000, 3)):
        src = rng.integers(1, n + 1, n * deg).astype(np.int32)
        dst = rng.integers(1, n + 1, n * deg).astype(np.int32)
        acc = (rng.random(n) < 0.05).astype(np.uint8)
        g = synth.Graph(n=n, src=src, dst=dst, acc=acc, name=f"dense{n}x{deg}")
        csr = mc.build_csr(g.n, g.src, g.dst)
        check_detect(mc, g, csr, flags=mc.MAP_FLAG_STREAM | mc.MAP_FLAG_DIRECTION)
        check_propagate_all(mc, g, csr, max_k=3, flags=mc.MAP_FLAG_STREAM | mc.MAP_FLAG_DIRECTION)
    g = hub_graph()
    csr = mc.build_csr(g.n, g.src, g.dst)
    check_detect(mc, g, csr, flags=mc.MAP_FLAG_STREAM | mc.MAP_FLAG_DIRECTION)
    check_propagate_all(mc, g, csr, max_k=2, flags=mc.MAP_FLAG_STREAM | mc.MAP_FLAG_DIRECTION)


def test_direction_switch_needs_transposed(mc):
    g = synth.config1()
    csr = mc.build_csr(g.n, g.src, g.dst, transposed=False)
    with pytest.raises(mc.MapError):
        mc.detect(csr, g.acc, flags=mc.MAP_FLAG_DIRECTION)


@pytest.mark.parametrize("n,planted", [(1 << 14, False), (1 << 14, True), (1 << 16, False), (1 << 16, True)])
def test_config2_reduced(mc, n, planted):
    g = synth.config2(seed=2, n=n, planted=planted)
    csr = mc.build_csr(g.n, g.src, g.dst)
    _, ref = check_detect(mc, g, csr)
    if planted:
        assert ref.found == 1
    check_detect(mc, g, csr, flags=mc.MAP_FLAG_PUSH, ref=ref)


def test_config3_reduced(mc):
    g = synth.config3(n=1 << 18)
    csr = mc.build_csr(g.n, g.src, g.dst)
    _, ref = check_detect(mc, g, csr)
    check_propagate_all(mc, g, csr, max_k=2)
    check_detect(mc, g, csr, flags=mc.MAP_FLAG_PUSH, ref=ref)
    check_detect(mc, g, csr, flags=mc.MAP_FLAG_STREAM | mc.MAP_FLAG_DIRECTION, ref=ref)


@pytest.mark.parametrize("g", [c for c in _random_cases() if c.n >= 64] + [synth.config1(), synth.config1(dag=True),
                               synth.config2(seed=4, n=1 << 15)], ids=lambda g: g.name)
@pytest.mark.parametrize("mode", ["sync", "sync+stream", "push"])
def test_barrier_per_sweep(mc, g, mode):
    """The same results with a grid barrier after every sweep (no asynchronous
    sweeps), and with frontier rounds over the transposed CSR."""
    if mode == "push":
        flags = mc.MAP_FLAG_PUSH
    else:
        flags = mc.MAP_FLAG_SYNC_SWEEPS | (mc.MAP_FLAG_STREAM if "stream" in mode else 0)
    csr = mc.build_csr(g.n, g.src, g.dst)
    check_detect(mc, g, csr, flags=flags)
    ref = oracle.map_detect(g, mode="desc", maps_cap=1)
    got, res = mc.propagate(csr, g.acc, flags=flags)
    assert res.status == 0 and np.array_equal(got.cpu().numpy(), ref.maps[0])


def test_push_edge_cases_and_flags(mc):
    """Frontier rounds on degenerate graphs; the flag needs the transposed CSR;
    MAP_FLAG_DENSE_ONLY overrides it."""
    cases = [synth.from_edges(1, [], [1], "n1-acc"), synth.from_edges(1, [(1, 1)], [1], "n1-loop"),
             synth.from_edges(300, [], [5, 17, 299], "no-edges"),
             synth.from_edges(5, [(1, 2), (2, 3), (3, 1), (3, 4), (4, 5)], [2, 4, 5], "hand"),
             synth.from_edges(6, [(1, 2), (2, 1), (1, 2), (3, 3), (4, 5), (5, 6), (6, 4)], [1, 2, 3, 6], "dups")]
    for g in cases:
        check_detect(mc, g, flags=mc.MAP_FLAG_PUSH)
        check_detect(mc, g, flags=mc.MAP_FLAG_PUSH | mc.MAP_FLAG_DENSE_ONLY)
    g = synth.config1()
    csr = mc.build_csr(g.n, g.src, g.dst, transposed=False)
    with pytest.raises(mc.MapError) as e:
        mc.detect(csr, g.acc, flags=mc.MAP_FLAG_PUSH)
    assert e.value.status == mc.MAP_EINVAL


# ------------------------------------------------------------- edge cases

def test_single_vertex_cases(mc):
    for edges, acc, want in [([], [], (0, 0, 0)), ([], [1], (0, 0, 1)), ([(1, 1)], [1], (1, 1, 1)),
                             ([(1, 1)], [], (0, 0, 0))]:
        g = synth.from_edges(1, edges, acc, f"n1{edges}{acc}")
        out, _ = check_detect(mc, g)
        assert out.result.verdict == want


def test_no_edges(mc):
    g = synth.from_edges(300, [], [5, 17, 299], "no-edges")
    out, _ = check_detect(mc, g)
    assert out.result.verdict == (0, 0, 1)


def test_all_accepting_and_duplicates(mc):
    rng = np.random.default_rng(3)
    n = 5000
    src = rng.integers(1, n + 1, 4000)
    dst = np.minimum(src + rng.integers(0, 3, 4000), n)
    src = np.concatenate([src, src[:1000]])  # duplicates
    dst = np.concatenate([dst, dst[:1000]])
    g = synth.Graph(n=n, src=src.astype(np.int32), dst=dst.astype(np.int32), acc=np.ones(n, np.uint8), name="allacc")
    check_detect(mc, g)


def hub_graph(n=200_000, seed=4):
    """One out-hub of 100,000 edges spanning many staged chunks, one in-hub,
    a chain, and 300 accepting vertices."""
    rng = np.random.default_rng(seed)
    hub_out = np.stack([np.full(100_000, 7), rng.integers(1, n + 1, 100_000)], 1)
    hub_in = np.stack([rng.integers(1, n + 1, 50_000), np.full(50_000, 150_000)], 1)
    chain = np.stack([np.arange(1000, 1500), np.arange(1001, 1501)], 1)
    e = np.concatenate([hub_out, hub_in, chain]).astype(np.int32)
    acc = np.zeros(n, np.uint8)
    acc[rng.choice(n, 300, replace=False)] = 1
    acc[150_000 - 1] = 1
    return synth.Graph(n=n, src=e[:, 0].copy(), dst=e[:, 1].copy(), acc=acc, name="hubs")


@pytest.mark.parametrize("flags", [0, 0x4, 0x4 | 0x40, 0x8], ids=["auto", "stream", "stream-async", "sync"])
def test_hub_rows_all_modes(mc, flags):
    """The hub graph in every sweep mode: streamed tiles fold the hub row with
    the whole wave (filtered and asynchronous), barrier mode per lane."""
    g = hub_graph()
    csr = mc.build_csr(g.n, g.src, g.dst)
    check_detect(mc, g, csr, flags=flags)
    check_propagate_all(mc, g, csr, max_k=2, flags=flags)


def test_hub_star_mix(mc):
    """A config-3 style DAG with three out-hubs of 10^5 edges each and an
    in-hub, streamed (every block streams at this size)."""
    base = synth.config3(n=1 << 21)
    rng = np.random.default_rng(9)
    hubs = []
    for h in (1 << 20, (1 << 21) - 5, 3 << 19):
        hubs.append(np.stack([np.full(100_000, h), rng.integers(1, h, 100_000)], 1))
    hubs.append(np.stack([rng.integers(1 << 20, 1 << 21, 30_000), np.full(30_000, 12345)], 1))
    e = np.concatenate([np.stack([base.src, base.dst], 1)] + hubs).astype(np.int32)
    acc = base.acc.copy()
    acc[[12345 - 1, 999 - 1]] = 1
    g = synth.Graph(n=base.n, src=e[:, 0].copy(), dst=e[:, 1].copy(), acc=acc, name="hub-star-mix")
    csr = mc.build_csr(g.n, g.src, g.dst)
    check_detect(mc, g, csr)
    check_detect(mc, g, csr, flags=mc.MAP_FLAG_NO_FILTER)


def test_hub_rows(mc):
    # one out-hub spanning many LDS chunks, one in-hub, plus a chain
    n = 200_000
    rng = np.random.default_rng(4)
    hub_out = np.stack([np.full(100_000, 7), rng.integers(1, n + 1, 100_000)], 1)
    hub_in = np.stack([rng.integers(1, n + 1, 50_000), np.full(50_000, 150_000)], 1)
    chain = np.stack([np.arange(1000, 1500), np.arange(1001, 1501)], 1)
    e = np.concatenate([hub_out, hub_in, chain]).astype(np.int32)
    acc = np.zeros(n, np.uint8)
    acc[rng.choice(n, 300, replace=False)] = 1
    acc[150_000 - 1] = 1
    g = synth.Graph(n=n, src=e[:, 0].copy(), dst=e[:, 1].copy(), acc=acc, name="hubs")
    csr = mc.build_csr(g.n, g.src, g.dst)
    check_detect(mc, g, csr)
    check_propagate_all(mc, g, csr, max_k=2)


@pytest.mark.parametrize("k", [2, 50, 200])
def test_increasing_chain(mc, k):
    g = synth.from_edges(k, [(i, i + 1) for i in range(1, k)], range(1, k + 1), f"chain{k}")
    out, _ = check_detect(mc, g)
    assert out.result.verdict == (0, 0, k)


def test_star_graphs(mc):
    n = 10_000
    out_star = [(1, v) for v in range(2, n + 1)]
    in_star = [(v, 1) for v in range(2, n + 1)]
    for edges, name in ((out_star, "out-star"), (in_star, "in-star"), (out_star + [(n, 1)], "star+back")):
        g = synth.from_edges(n, edges, range(1, n + 1, 97), name)
        check_detect(mc, g)


def test_trace_cap_and_iteration_cap(mc):
    k = 40
    g = synth.from_edges(k, [(i, i + 1) for i in range(1, k)], range(1, k + 1), "chain-cap")
    check_detect(mc, g, trace_cap=5)
    out, ref = check_detect(mc, g, max_iterations=7)
    assert out.result.status == mc.MAP_ENOTCONVERGED and out.result.iterations == 7


def test_no_digest_flag(mc):
    g = synth.config1(dag=True)
    out, _ = check_detect(mc, g, flags=mc.MAP_FLAG_NO_TRACE_DIGEST)
    assert np.all(out.trace[:, 2] == 0)


# ---------------------------------------------------------------- CSR build

def _stable_csr(n, key, other):
    """Row pointer and columns of the CSR whose rows list their edges in
    edge-list order: a stable sort of the edges by key (numpy's)."""
    order = np.argsort(key, kind="stable")
    deg = np.bincount(key - 1, minlength=n)
    rp = np.concatenate([[0], np.cumsum(deg)])
    return rp, (other[order] - 1).astype(np.int32)


def test_csr_build_matches_edge_list(mc):
    g = synth.config2(seed=5, n=1 << 15, planted=True)
    csr = mc.build_csr(g.n, g.src, g.dst)
    assert int(csr.status.item()) == 0
    for rp, col, key, other in ((csr.row_ptr, csr.col, g.src, g.dst), (csr.rrow_ptr, csr.rcol, g.dst, g.src)):
        want_rp, want_col = _stable_csr(g.n, key, other)
        assert np.array_equal(rp.cpu().numpy(), want_rp)
        assert np.array_equal(col.cpu().numpy()[:g.m], want_col)


def _check_csr(csr, n, src, dst, orientations=2):
    """Both CSRs hold exactly the in-range edges (ids 1..n at both ends), each
    row in edge-list order."""
    ok = (src >= 1) & (src <= n) & (dst >= 1) & (dst <= n)
    src, dst = src[ok], dst[ok]
    pairs = ((csr.row_ptr, csr.col, src, dst), (csr.rrow_ptr, csr.rcol, dst, src))[:orientations]
    for rp, col, key, other in pairs:
        want_rp, want_col = _stable_csr(n, key, other)
        assert np.array_equal(rp.cpu().numpy(), want_rp)
        assert np.array_equal(col.cpu().numpy()[:len(key)], want_col)


@pytest.mark.parametrize("order", ["random", "grouped"])
def test_csr_build_row_order_every_length(mc, order):
    """Rows of every length class the ordering passes distinguish (one lane
    up to 16 edges, one wave up to 64, a workgroup in LDS up to 4096, chunked
    merges beyond), each boundary from both sides, with the edge list shuffled
    (slots reserved in schedule order) or grouped by key: every row in
    edge-list order, and a second build byte-identical."""
    import torch
    rng = np.random.default_rng(31 if order == "random" else 32)
    lengths = [0, 1, 2, 3, 15, 16, 17, 33, 63, 64, 65, 100, 1000, 4095, 4096, 4097, 8191, 8192, 8193, 20000,
               100_003]
    n = 5000
    rows = rng.permutation(np.arange(1, n + 1))[:len(lengths)]
    # shuffled lists of 2^20 edges or more take the radix path, grouped ones the per-row cursors
    key = np.concatenate([np.full(d, r, np.int32) for d, r in zip(lengths, rows)]
                         + [rng.integers(1, n + 1, 1_000_000).astype(np.int32)])
    other = rng.integers(1, n + 1, len(key)).astype(np.int32)
    perm = rng.permutation(len(key)) if order == "random" else np.argsort(key, kind="stable")
    src, dst = key[perm].copy(), other[perm].copy()
    print("csr row order", order, "n", n, "m", len(src), flush=True)
    csr = mc.build_csr(n, src, dst)
    assert int(csr.status.item()) == 0
    _check_csr(csr, n, src, dst)
    again = mc.build_csr(n, src, dst)
    for a, b in ((csr.row_ptr, again.row_ptr), (csr.col, again.col), (csr.rrow_ptr, again.rrow_ptr),
                 (csr.rcol, again.rcol)):
        assert torch.equal(a, b)


def _grouped(rng, n, max_deg, m_cap=None):
    """Edges grouped by source (generation order), degrees 0..max_deg."""
    deg = rng.integers(0, max_deg + 1, n)
    src = np.repeat(np.arange(1, n + 1, dtype=np.int32), deg)
    if m_cap is not None:
        src = src[:m_cap]
    dst = rng.integers(1, n + 1, len(src)).astype(np.int32)
    return src, dst


@pytest.mark.parametrize("case", ["random", "grouped", "hub", "ragged", "invalid", "invalid_random"])
def test_csr_build_key_runs(mc, case):
    """Edges with equal keys share one atomic per run of a wave: runs that
    cross wave boundaries, runs broken by out-of-range edges, lists in random
    order, a vertex whose edges fill many waves, a ragged tail."""
    rng = np.random.default_rng({"random": 11, "grouped": 12, "hub": 13, "ragged": 14, "invalid": 15,
                                 "invalid_random": 16}[case])
    n = 4000
    if case == "random":
        src = rng.integers(1, n + 1, 50_000).astype(np.int32)
        dst = rng.integers(1, n + 1, 50_000).astype(np.int32)
        src[1000:1100] = 7                       # one run among random keys
    elif case == "grouped":
        src, dst = _grouped(rng, n, 200)
    elif case == "hub":
        src, dst = _grouped(rng, n, 8)
        src = np.concatenate([src[:5000], np.full(70_000, 123, np.int32), src[5000:]])
        dst = np.concatenate([dst[:5000], rng.integers(1, n + 1, 70_000).astype(np.int32), dst[5000:]])
    elif case == "ragged":
        src, dst = _grouped(rng, n, 90, m_cap=64 * 1000 + 37)
    elif case == "invalid_random":
        # shuffled and over 2^20 edges (the radix path), with edges outside 1..n at either end
        src = rng.integers(1, n + 1, 1_100_000).astype(np.int32)
        dst = rng.integers(1, n + 1, 1_100_000).astype(np.int32)
        bad = rng.choice(len(src), 300, replace=False)
        src[bad[:100]] = n + 1
        dst[bad[100:200]] = 0
        src[bad[200:]] = -5
    else:
        src, dst = _grouped(rng, n, 150)
        bad = rng.choice(len(src), 300, replace=False)
        src[bad[:100]] = 0
        src[bad[100:200]] = n + 1
        dst[bad[200:]] = -3
    print("csr runs", case, "n", n, "m", len(src), flush=True)
    csr = mc.build_csr(n, src, dst)
    status = int(csr.status.item())
    assert status == (mc.MAP_ERANGE_DEV if case.startswith("invalid") else 0)
    _check_csr(csr, n, src, dst)


def test_csr_build_grid_stride(mc):
    """More edges than one pass of the launch covers (65,536 workgroups of 256
    threads), grouped by source, so runs also cross the stride boundary."""
    rng = np.random.default_rng(16)
    n = 1 << 20
    src, dst = _grouped(rng, n, 40)
    assert len(src) > 65536 * 256
    print("csr grid stride n", n, "m", len(src), flush=True)
    csr = mc.build_csr(n, src, dst, transposed=False)
    assert int(csr.status.item()) == 0
    _check_csr(csr, n, src, dst, orientations=1)


@pytest.mark.parametrize("order", ["shuffled", "grouped"])
def test_csr_build_rows_past_one_grid_pass(mc, order):
    """n = 2^25 vertices, more rows than one pass of the capped launch covers
    (65,536 workgroups of 256 threads = 2^24): keys spread over the whole
    range, many above 2^24, rows of every length class; shuffled (the radix
    path) or grouped by key (per-row cursors and row ordering)."""
    rng = np.random.default_rng(17)
    n = 1 << 25
    key = np.concatenate([rng.integers(1, n + 1, 600_000), rng.integers((1 << 24) + 1, n + 1, 600_000),
                          np.full(40, n), np.full(5000, n - 1), np.full(70, 1 << 24), np.full(70, (1 << 24) + 1)])
    other = rng.integers(1, n + 1, len(key))
    perm = rng.permutation(len(key)) if order == "shuffled" else np.argsort(key, kind="stable")
    src, dst = key[perm].astype(np.int32), other[perm].astype(np.int32)
    print("csr past one grid pass", order, "n", n, "m", len(src), flush=True)
    csr = mc.build_csr(n, src, dst)
    assert int(csr.status.item()) == 0
    _check_csr(csr, n, src, dst)


def test_csr_build_range_error(mc):
    import torch
    n = 10
    src = torch.tensor([1, 2, 11], dtype=torch.int32)
    dst = torch.tensor([2, 3, 1], dtype=torch.int32)
    csr = mc.build_csr(n, src, dst)
    torch.cuda.synchronize()
    assert int(csr.status.item()) == mc.MAP_ERANGE_DEV


def test_csr_build_empty(mc):
    csr = mc.build_csr(5, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert csr.row_ptr.cpu().numpy().tolist() == [0] * 6


# ------------------------------------------------------- schedule independence

def test_repeated_runs_identical(mc):
    g = synth.config2(seed=7, n=1 << 16)
    csr = mc.build_csr(g.n, g.src, g.dst)
    first = mc.detect(csr, g.acc, trace_cap=g.n_acc + 1)
    for _ in range(5):
        again = mc.detect(csr, g.acc, trace_cap=g.n_acc + 1)
        assert again.result.verdict == first.result.verdict
        assert np.array_equal(again.trace[:, [0, 2]], first.trace[:, [0, 2]])


# ------------------------------------------------------------------ full size

def _golden(key):
    path = os.path.join(ROOT, "tests", "golden", "full_size.json")
    data = json.load(open(path))
    if key not in data:
        pytest.fail(f"golden {key} missing: run tests/golden/make_goldens.py")
    return data[key]


def _check_golden(mc, g, gold):
    import hashlib
    say("full-size detect", g.name, "m", g.m)
    assert g.n == gold["n"] and g.m == gold["m"]
    csr = mc.build_csr(g.n, g.src, g.dst)
    out = mc.detect(csr, g.acc, trace_cap=g.n_acc + 1, want_acc=True)
    r = out.result
    assert r.status == 0
    assert r.verdict == (gold["found"], gold["witness"], gold["iterations"])
    assert r.accepting_left == gold["accepting_left"]
    assert [int(x) for x in out.trace[:, 0]] == gold["dels"]
    dig = out.trace[:, 2].astype("<u8")
    assert [f"{int(x):016x}" for x in dig[:8]] == gold["digest_head"]
    assert hashlib.sha256(dig.tobytes()).hexdigest() == gold["digest_sha256"]
    return csr, out


@pytest.mark.parametrize("key,planted", [("c2B", False), ("c2A", True)])
def test_config2_full_size(mc, key, planted):
    g = synth.config2(planted=planted)
    csr, out = _check_golden(mc, g, _golden(key))
    # first iteration's full map vector against the oracle's fixpoint
    got, res = mc.propagate(csr, g.acc)
    want, _ = oracle.fixpoint(g, mode="desc")
    assert np.array_equal(got.cpu().numpy(), want)


@pytest.mark.parametrize("direction", [False, True], ids=["pull", "direction-switch"])
def test_config3_literal_full_size(mc, direction):
    """Config 3's literal reading: the config-1 generator at 2^25 vertices with
    the edges s > d kept (a DAG of about 42M edges, 5% accepting), against the
    oracle's golden; with filtered pull sweeps and with the direction switch."""
    import hashlib
    g = synth.config1(seed=3, n=1 << 25, dag=True)
    gold = _golden("c3lit")
    assert g.n == gold["n"] and g.m == gold["m"]
    say("full-size detect", g.name, "m", g.m, "direction", direction)
    csr = mc.build_csr(g.n, g.src, g.dst, transposed=direction)
    out = mc.detect(csr, g.acc, trace_cap=gold["iterations"] + 1,
                    flags=mc.MAP_FLAG_DIRECTION if direction else 0)
    r = out.result
    assert r.status == 0
    assert r.verdict == (gold["found"], gold["witness"], gold["iterations"])
    assert r.accepting_left == gold["accepting_left"]
    assert [int(x) for x in out.trace[:, 0]] == gold["dels"]
    dig = out.trace[:, 2].astype("<u8")
    assert hashlib.sha256(dig.tobytes()).hexdigest() == gold["digest_sha256"]


def test_config3_full_size(mc):
    g = synth.config3()
    csr, _ = _check_golden(mc, g, _golden("c3"))
    # the generator lists edges by source, so the pull CSR in edge order is
    # the destination column as it stands
    assert np.all(np.diff(g.src) >= 0)
    assert np.array_equal(csr.col.cpu().numpy()[:g.m], g.dst - 1)
