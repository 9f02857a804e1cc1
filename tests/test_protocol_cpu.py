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
of the propagation (computed here by plain iteration).  In the first models
released writes become visible at once (sequential consistency), which pins
the logic of the protocol.  Two planted mistakes (reporting quiet from the
counter value read at the end of the sweep instead of its start; bumping the
counter before releasing the writes) must be caught.

A later model splits each workgroup into waves whose stores travel through
the memory system (in flight, completed in the XCD's L2, written back), so
that the release the device performs is modelled too: every wave completes
its stores before the workgroup barrier and the leader writes back; the
earlier leader-only wait must be caught.  A last model pins the bound on
asynchronous sweeping: a livelocked block ends the launch.
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


# ------------------------------------------- per-wave visibility of stores
#
# The device side of a release.  A workgroup's rows are split among its
# waves; a wave's store to memory is first in flight, then completes (is
# acknowledged by the L2 of the workgroup's XCD), and is visible to other XCDs
# only once an L2 write-back covers it (or the line is evicted).  A wave waits
# for its own stores to complete with `s_waitcnt vmcnt(0)`; the leader's
# agent-scope release writes back the completed lines of its L2, then the
# leader bumps the change counter.  Readers on other XCDs see memory.
#
# The kept protocol: every wave completes its stores before the workgroup
# barrier, the leader then writes back and bumps.  The planted slip is the
# earlier build's: only the leader's wave waits for its own stores, so another
# wave's store may still be in flight when the leader writes back and bumps.
# The check is on the rows' own values when done is declared: every block's
# rows must hold the least fixpoint.

class Mem:
    def __init__(self, n, nb):
        self.mem = [0] * n                     # what other XCDs read
        self.inflight = []                     # (block, v, value): issued, not yet in L2
        self.l2 = [dict() for _ in range(nb)]  # per block: completed, not written back
        self.dirty = 0
        self.quiet = [None] * nb
        self.done = False
        self.clock = 0
        self.abort = False

    def complete(self, idx):
        b, v, x = self.inflight.pop(idx)
        self.l2[b][v] = max(self.l2[b].get(v, 0), x)

    def writeback(self, b):
        for v, x in self.l2[b].items():
            self.mem[v] = max(self.mem[v], x)
        self.l2[b].clear()


def wave_block(b, rows, nwaves, succ, acc, sh, leader_only, bound=None, stuck=False):
    """One block of `nwaves` waves as a generator; rows are cut among the waves."""
    own = {v: 0 for v in rows}
    cuts = [rows[0] + round(i * len(rows) / nwaves) for i in range(nwaves + 1)] if rows else [0] * (nwaves + 1)
    wave_of = {v: i for i in range(nwaves) for v in range(cuts[i], cuts[i + 1])}
    d_seen = None
    first = True
    t_iter = sh.clock
    while True:
        if not first:
            while True:
                if sh.done or sh.abort:
                    return
                if bound is not None and sh.clock - t_iter > bound:
                    sh.abort = True                  # the launch ends with MAP_EDEVICE
                    return
                d = sh.dirty
                yield
                if d != d_seen:
                    break
                if b == 0:
                    want = (1, d + 1)
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
        mine = []                                    # (wave, v, value) stored by this sweep
        for v in rows:
            best = own[v]
            for w in succ[v]:
                x = own[w] if w in own else sh.mem[w]
                yield
                best = max(best, x, (w + 1) if acc[w] else 0)
            if best > own[v]:
                own[v] = best
                changed = True
                sh.inflight.append((b, v, best))     # the wave's store, now in flight
                mine.append(wave_of[v])
        if stuck:
            changed = True                           # a block that never settles (livelock)
        if changed:
            # every wave (or, with the slip, only the leader's wave 0) waits
            # for its stores to complete; then the workgroup barrier
            waits = range(nwaves) if not leader_only else [0]
            for wv in waits:
                i = 0
                while i < len(sh.inflight):
                    bb, v, _ = sh.inflight[i]
                    if bb == b and wave_of[v] == wv:
                        sh.complete(i)
                    else:
                        i += 1
            yield
            sh.writeback(b)                          # the leader's agent-scope release
            yield
            sh.dirty += 1
            d_seen = None
        else:
            sh.quiet[b] = (1, d0 + 1)
            d_seen = d0
        yield


def _wave_block_values(n, succ, acc, nb, nwaves, seed, **kw):
    """Runs the model and returns (shared state, the rows' values at the end)."""
    rng = random.Random(seed)
    sh = Mem(n, nb)
    cuts = [round(i * n / nb) for i in range(nb + 1)]
    owns = [dict() for _ in range(nb)]

    def track(b, gen):
        # mirror the block's own copy as it runs: read it out of the frame
        while True:
            try:
                next(gen)
            except StopIteration:
                return
            owns[b].update(gen.gi_frame.f_locals["own"]) if gen.gi_frame else None
            yield

    bound, stuck_block = kw.get("bound"), kw.get("stuck_block")
    gens = [track(b, wave_block(b, list(range(cuts[b], cuts[b + 1])), nwaves, succ, acc, sh,
                                kw.get("leader_only", False), bound, stuck=(b == stuck_block)))
            for b in range(nb)]
    live = list(range(nb))
    steps = 0
    while live:
        sh.clock += 1
        r = rng.random()
        if sh.inflight and r < 0.05:
            sh.complete(rng.randrange(len(sh.inflight)))
        elif r < 0.07:
            sh.writeback(rng.randrange(nb))
        i = rng.choice(live)
        try:
            next(gens[i])
        except StopIteration:
            live.remove(i)
        steps += 1
        if steps >= kw.get("max_steps", 400_000):
            return sh, None
    vals = [0] * n
    for o in owns:
        for v, x in o.items():
            vals[v] = x
    return sh, vals


def _chain(n, down=False):
    """A chain crossing every block boundary.  Up: v -> v+1, the last vertex
    accepting (the rows other blocks read are the first row of each block, in
    wave 0).  Down: v -> v-1, vertex 0 accepting (they are the last row of
    each block, in the last wave)."""
    if down:
        return [[v - 1] if v > 0 else [] for v in range(n)], [True] + [False] * (n - 1)
    return [[v + 1] if v + 1 < n else [] for v in range(n)], [False] * (n - 1) + [True]


@pytest.mark.parametrize("seed", range(25))
def test_every_wave_completes_its_stores(seed):
    """Kept protocol: done is declared only at the least fixpoint, whatever the
    memory system does with stores in flight and dirty L2 lines."""
    rng = np.random.default_rng(3000 + seed)
    n = int(rng.integers(4, 16))
    nb = int(rng.integers(2, min(n, 4) + 1))
    succ, acc = random_graph(rng, n, 3, 0.3)
    want = least_fixpoint(n, succ, acc)
    for s in range(4):
        sh, vals = _wave_block_values(n, succ, acc, nb, 2, seed * 10 + s)
        assert sh.done and not sh.abort
        assert vals == want, (seed, s)


@pytest.mark.parametrize("down", [False, True])
def test_chain_with_waves(down):
    n, nb = 16, 4
    succ, acc = _chain(n, down)
    want = least_fixpoint(n, succ, acc)
    for s in range(40):
        sh, vals = _wave_block_values(n, succ, acc, nb, 2, s)
        assert sh.done and vals == want


def test_planted_leader_only_release_is_caught():
    """The leader's release covering only its own wave's stores lets done be
    declared while a row of another block still misses a value (the rows the
    next block reads are stored by the last wave of each block)."""
    n, nb = 16, 4
    succ, acc = _chain(n, down=True)
    want = least_fixpoint(n, succ, acc)
    wrong = 0
    for s in range(300):
        sh, vals = _wave_block_values(n, succ, acc, nb, 2, s, leader_only=True)
        wrong += sh.done and vals != want
    assert wrong > 0


# ------------------------------------------------ bound on async sweeping
#
# A fixpoint computation whose sweeping has not settled within a bound of
# device wall clock ends the launch (MAP_EDEVICE), however often the change
# counter moves.  A block that never settles (a livelock, e.g. a word that is
# not what its owner wrote) must end every block's loop; a bound far above a
# normal run's length is never hit.

def test_normal_runs_stay_within_the_bound():
    rng = np.random.default_rng(4000)
    for seed in range(20):
        n = int(rng.integers(4, 14))
        nb = int(rng.integers(2, min(n, 4) + 1))
        succ, acc = random_graph(rng, n, 3, 0.3)
        sh, vals = _wave_block_values(n, succ, acc, nb, 2, seed, bound=200_000)
        assert sh.done and not sh.abort
        assert vals == least_fixpoint(n, succ, acc)


@pytest.mark.parametrize("stuck_block", [0, 2])
def test_livelock_ends_at_the_bound(stuck_block):
    n, nb = 12, 3
    succ, acc = _chain(n)
    sh, vals = _wave_block_values(n, succ, acc, nb, 2, 7, bound=3_000, stuck_block=stuck_block,
                                  max_steps=200_000)
    assert vals is not None, "the bound did not end the livelocked run"
    assert sh.abort and not sh.done


def test_livelock_without_the_bound_runs_on():
    """Without the bound (the earlier per-wait limit restarted whenever the
    counter moved) the same livelock never ends."""
    n, nb = 12, 3
    succ, acc = _chain(n)
    sh, vals = _wave_block_values(n, succ, acc, nb, 2, 7, bound=None, stuck_block=1, max_steps=50_000)
    assert vals is None and not sh.abort
