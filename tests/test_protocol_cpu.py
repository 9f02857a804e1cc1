"""Models of the loop kernel's cross-workgroup protocols (the asynchronous
fixpoint control, the iteration parity of packed words, the barrier reduction
sets), run under random interleavings on the CPU (no GPU, no library).

The model follows the kernel's protocol step by step:

* each block owns a contiguous range of rows and is the only writer of them;
  its writes stay private until it releases them;
* a sweep reads the change counter d0 first; it then reads successors' values
  one at a time, interleaved with every other block's steps (each read sees
  whatever has been released so far);
* a sweep that raised a row releases its writes and then bumps the counter; a
  sweep that changed nothing reports quiet (iteration, d0 + 1);
* a block sweeps again whenever the counter differs from the value its last
  quiet sweep started from;
* block 0 declares the fixpoint when every block's report equals
  (iteration, counter + 1) and a re-read of the counter is unchanged.

Whenever done is declared, the released values must equal the least fixpoint
of the propagation (computed here by plain iteration).  Released writes
become visible at once (sequential consistency), so the model pins the logic
of the protocol, not the ordering the fences give on the device.  Two planted
mistakes (reporting quiet from the counter
value read at the end of the sweep instead of its start; bumping the counter
before releasing the writes) must be caught.
"""
import random

import numpy as np
import pytest


def least_fixpoint(n, succ, acc):
    """map(v) = max over successors w of max(acc(w) * (w + 1), map(w)), by iteration."""
    val = [0] * n
    changed = True
    while changed:
        changed = False
        for v in range(n):
            b = val[v]
            for w in succ[v]:
                b = max(b, val[w], (w + 1) if acc[w] else 0)
            if b > val[v]:
                val[v] = b
                changed = True
    return val


class Shared:
    def __init__(self, n, nb):
        self.val = [0] * n           # released values
        self.dirty = 0
        self.quiet = [None] * nb
        self.done = False


def block(b, rows, succ, acc, sh, nb, tag, late_d0, bump_first):
    """One block as a generator: every yield is a point where other blocks may run."""
    own = {v: 0 for v in rows}           # this block's current (possibly unreleased) values
    d_seen = None
    first = True
    while True:
        if not first:
            # poll: stop when done, sweep when the counter moved
            while True:
                if sh.done:
                    return
                d = sh.dirty
                yield
                if d != d_seen:
                    break
                if b == 0:
                    want = (tag, d + 1)
                    if all(q == want for q in sh.quiet):
                        yield
                        if sh.dirty == d:
                            sh.done = True
                            return
                yield
        first = False
        d0 = sh.dirty
        yield
        changed = False
        for v in rows:
            best = own[v]
            for w in succ[v]:
                x = own[w] if w in own else sh.val[w]     # own rows from the block's own copy
                yield
                best = max(best, x, (w + 1) if acc[w] else 0)
            if best > own[v]:
                own[v] = best
                changed = True
        if changed:
            if bump_first:                               # planted mistake: counter before release
                sh.dirty += 1
                yield
            for v in rows:                               # release
                sh.val[v] = own[v]
            yield
            if not bump_first:
                sh.dirty += 1
            d_seen = None
        else:
            if late_d0:
                d0 = sh.dirty                            # the planted mistake
            sh.quiet[b] = (tag, d0 + 1)
            d_seen = d0
        yield


def run(n, succ, acc, nb, seed, late_d0=False, bump_first=False, max_steps=2_000_000):
    rng = random.Random(seed)
    sh = Shared(n, nb)
    cuts = [round(i * n / nb) for i in range(nb + 1)]
    gens = [block(b, list(range(cuts[b], cuts[b + 1])), succ, acc, sh, nb, 1, late_d0, bump_first)
            for b in range(nb)]
    live = list(range(nb))
    steps = 0
    while live:
        i = rng.choice(live)
        try:
            next(gens[i])
        except StopIteration:
            live.remove(i)
        steps += 1
        assert steps < max_steps, "the model did not terminate"
    return sh


def random_graph(rng, n, deg, p_acc):
    succ = [sorted(set(rng.integers(0, n, rng.integers(0, deg + 1)).tolist())) for _ in range(n)]
    acc = (rng.random(n) < p_acc).tolist()
    return succ, acc


@pytest.mark.parametrize("seed", range(40))
def test_done_only_at_the_fixpoint(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 14))
    nb = int(rng.integers(2, min(n, 5) + 1))
    succ, acc = random_graph(rng, n, 3, 0.3)
    want = least_fixpoint(n, succ, acc)
    for s in range(5):
        sh = run(n, succ, acc, nb, seed * 100 + s)
        assert sh.done
        assert sh.val == want, (seed, s)


def test_chain_across_blocks():
    """A chain whose values cross every block boundary, in the worst direction."""
    n, nb = 12, 4
    succ = [[v + 1] if v + 1 < n else [] for v in range(n)]
    acc = [False] * (n - 1) + [True]
    want = least_fixpoint(n, succ, acc)
    assert want == [n] * (n - 1) + [0]
    for s in range(30):
        sh = run(n, succ, acc, nb, s)
        assert sh.val == want


@pytest.mark.parametrize("mistake", ["late_d0", "bump_first"])
def test_planted_mistake_is_caught(mistake):
    """Two plausible slips in the protocol must let done be declared before
    the fixpoint in some interleaving: reporting quiet from the counter read
    at the end of a sweep, and bumping the counter before releasing the
    writes."""
    n, nb = 12, 4
    succ = [[v + 1] if v + 1 < n else [] for v in range(n)]
    acc = [False] * (n - 1) + [True]
    want = least_fixpoint(n, succ, acc)
    wrong = 0
    for s in range(300):
        sh = run(n, succ, acc, nb, s, **{mistake: True})
        wrong += sh.val != want
    assert wrong > 0


# ----------------------------------------------------- two outer iterations
#
# Packed words carry the iteration parity: a word of the other parity reads
# as 0, and the first sweep of an iteration (the reset) takes what the
# accepting successors send (their ids) instead of reading values.  The model
# runs iteration 1 to its fixpoint, strips, and starts iteration 2 on the
# words iteration 1 left (blocks begin their resets at different times).

def block_iter(b, rows, succ, acc, sh, tag, par, ignore_parity=False):
    def sent(word, w):
        p, a, m = word
        if p != par and not ignore_parity:
            return 0
        return max(m, w + 1) if a else m

    own = {}
    d_seen = None
    first = True
    while True:
        if not first:
            while True:
                if sh.done == tag:
                    return
                d = sh.dirty
                yield
                if d != d_seen:
                    break
                if b == 0:
                    want = (tag, d + 1)
                    if all(q == want for q in sh.quiet):
                        yield
                        if sh.dirty == d:
                            sh.done = tag
                            return
                yield
        d0 = sh.dirty
        yield
        changed = False
        for v in rows:
            if first:
                best = 0
                for w in succ[v]:
                    best = max(best, (w + 1) if acc[w] else 0)
                    yield
                own[v] = (par, acc[v], best)
                changed |= best != 0 or acc[v]
                continue
            best = own[v][2]
            for w in succ[v]:
                x = sent(own[w], w) if w in own else sent(sh.val[w], w)
                yield
                best = max(best, x)
            if best > own[v][2]:
                own[v] = (par, own[v][1], best)
                changed = True
        if first and not changed:
            # The reset writes every row; new words of value 0 read as the
            # stale ones do (0), so nothing needs announcing.
            for v in rows:
                sh.val[v] = own[v]
        first = False
        if changed:
            for v in rows:
                sh.val[v] = own[v]
            yield
            sh.dirty += 1
            d_seen = None
        else:
            sh.quiet[b] = (tag, d0 + 1)
            d_seen = d0
        yield


def run_iter(sh, n, succ, acc, nb, seed, tag, ignore_parity=False):
    rng = random.Random(seed)
    cuts = [round(i * n / nb) for i in range(nb + 1)]
    par = tag & 1
    gens = [block_iter(b, list(range(cuts[b], cuts[b + 1])), succ, acc, sh, tag, par, ignore_parity)
            for b in range(nb)]
    live = list(range(nb))
    steps = 0
    while live:
        i = rng.choice(live)
        try:
            next(gens[i])
        except StopIteration:
            live.remove(i)
        steps += 1
        assert steps < 2_000_000, "the model did not terminate"
    assert all(p == par for (p, _, _) in sh.val), "a row missed its reset"
    return [m for (_, _, m) in sh.val]


@pytest.mark.parametrize("seed", range(30))
def test_second_iteration_reads_stale_words_as_zero(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(3, 14))
    nb = int(rng.integers(2, min(n, 5) + 1))
    succ, acc1 = random_graph(rng, n, 3, 0.4)
    want1 = least_fixpoint(n, succ, acc1)
    # the strip between the iterations: every accepting vertex that is some
    # vertex's map value loses its flag
    acc2 = list(acc1)
    for m in want1:
        if m:
            acc2[m - 1] = False
    want2 = least_fixpoint(n, succ, acc2)
    for s in range(4):
        sh = Shared(n, nb)
        sh.val = [(0, False, 0)] * n
        sh.done = 0
        got1 = run_iter(sh, n, succ, acc1, nb, seed * 10 + s, 1)
        assert got1 == want1
        sh.quiet = [None] * nb
        got2 = run_iter(sh, n, succ, acc2, nb, seed * 10 + s + 5, 2)
        assert got2 == want2, (seed, s)


def test_planted_parity_slip_is_caught():
    """Reading a word of the previous iteration as a value lets stale values
    into the next fixpoint in some interleaving."""
    wrong = 0
    for seed in range(60):
        rng = np.random.default_rng(2000 + seed)
        n = int(rng.integers(4, 14))
        nb = int(rng.integers(2, min(n, 5) + 1))
        succ, acc1 = random_graph(rng, n, 3, 0.4)
        want1 = least_fixpoint(n, succ, acc1)
        acc2 = list(acc1)
        for m in want1:
            if m:
                acc2[m - 1] = False
        want2 = least_fixpoint(n, succ, acc2)
        sh = Shared(n, nb)
        sh.val = [(0, False, 0)] * n
        sh.done = 0
        run_iter(sh, n, succ, acc1, nb, seed, 1)
        sh.quiet = [None] * nb
        wrong += run_iter(sh, n, succ, acc2, nb, seed + 7, 2, ignore_parity=True) != want2
    assert wrong > 0


# ------------------------------------------------- barrier reduction epochs
#
# Counts reduced at a grid barrier go to one of three sets: epoch E adds into
# set E % 3; after barrier E every block reads set E % 3 (before it arrives at
# barrier E + 1); block 0 then clears set (E + 2) % 3, the one read during
# epoch E - 1 and next written in epoch E + 2.  The model checks every read
# sum under random interleavings, and that clearing the set of the next epoch
# instead is caught.

def reducer(b, nb, epochs, contrib, sh, clear_next):
    for e in range(epochs):
        sh.sets[e % 3] += contrib[b][e]             # atomic add
        yield
        sh.arrived[e] += 1                          # arrive at barrier e
        while sh.arrived[e] < nb:
            yield
        if b == 0:
            sh.sets[((e + 1) if clear_next else (e + 2)) % 3] = 0
        yield
        sh.reads.append((e, sh.sets[e % 3]))        # the reduced value
        yield


@pytest.mark.parametrize("clear_next", [False, True])
def test_barrier_reduction_sets(clear_next):
    wrong = 0
    for seed in range(200):
        rng = random.Random(seed)
        nb, epochs = rng.randint(2, 5), 6
        contrib = [[rng.randint(0, 9) for _ in range(epochs)] for _ in range(nb)]
        want = [sum(contrib[b][e] for b in range(nb)) for e in range(epochs)]

        class S:
            pass
        sh = S()
        sh.sets = [0, 0, 0]
        sh.arrived = [0] * epochs
        sh.reads = []
        gens = [reducer(b, nb, epochs, contrib, sh, clear_next) for b in range(nb)]
        live = list(range(nb))
        while live:
            i = rng.choice(live)
            try:
                next(gens[i])
            except StopIteration:
                live.remove(i)
        wrong += any(v != want[e] for e, v in sh.reads)
    if clear_next:
        assert wrong > 0
    else:
        assert wrong == 0
