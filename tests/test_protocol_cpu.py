"""A model of the asynchronous fixpoint control of the loop kernel, run under
random interleavings on the CPU (no GPU, no library).

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
