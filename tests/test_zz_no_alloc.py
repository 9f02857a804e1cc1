"""map_detect_noalloc (fixed device scratch, no allocation) against map_detect
(caller workspace), through the C ABI.

Two calls in a row on the shared scratch, the second with a smaller graph,
each compared field by field with map_detect on the same inputs: verdict, K,
witness, status, accepting set at exit, and the trace's removal counts and
map digests (the sweep counts depend on the schedule and are only checked to
be positive).  Both must also equal the oracle's verdict.
"""
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


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_both(mc, g, flags=0):
    import torch
    say("noalloc", g.name, "n", g.n, "m", g.m, "flags", flags)
    csr = mc.build_csr(g.n, g.src, g.dst, transposed=False)
    dev = csr.row_ptr.device
    acc = torch.from_numpy(g.acc).to(dev)
    cap = g.n_acc + 1
    outs = []
    for noalloc in (False, True):
        res = mc.new_result(dev)
        trace = torch.zeros((cap, 3), dtype=torch.int64, device=dev)
        acc_out = torch.zeros(g.n, dtype=torch.uint8, device=dev)
        if noalloc:
            rc = mc.map_detect_noalloc(g.n, csr.row_ptr, csr.col, acc, res, trace, acc_out, 0, flags)
        else:
            ws = mc.workspace(g.n, g.m)
            rc = mc.map_detect(g.n, csr.row_ptr, csr.col, None, None, acc, res, trace, acc_out, 0, flags, ws)
        assert rc == mc.MAP_OK, mc.strerror(rc)
        r = mc.Result.from_tensor(res)
        rows = min(r.iterations, cap)
        outs.append((r, trace.cpu().numpy().view(np.uint64)[:rows].copy(), acc_out.cpu().numpy()))
    (ra, ta, aa), (rb, tb, ab) = outs
    assert (rb.found, rb.witness, rb.iterations, rb.status, rb.accepting_left) == \
        (ra.found, ra.witness, ra.iterations, ra.status, ra.accepting_left)
    assert np.array_equal(tb[:, 0], ta[:, 0]) and np.array_equal(tb[:, 2], ta[:, 2])
    assert np.all(tb[:, 1] >= 1)
    assert np.array_equal(ab, aa)
    ref = oracle.map_detect(g)
    assert rb.verdict == ref.verdict
    say("  found", rb.found, "witness", rb.witness, "K", rb.iterations)
    return rb


def test_two_calls_second_smaller(mc):
    run_both(mc, synth.config2(seed=2, n=1 << 16, planted=True))
    run_both(mc, synth.config1(dag=True))


def test_modes_and_sizes(mc):
    # barrier-per-sweep and streamed sweeps on the shared scratch, then the
    # largest graph the scratch holds, then a tiny one
    run_both(mc, synth.config2(seed=3, n=1 << 15), flags=mc.MAP_FLAG_SYNC_SWEEPS)
    run_both(mc, synth.config2(seed=3, n=1 << 15), flags=mc.MAP_FLAG_STREAM)
    run_both(mc, synth.config1(seed=4, n=mc.MAP_NOALLOC_MAX_N))
    run_both(mc, synth.from_edges(5, [(1, 2), (2, 3), (3, 1), (3, 4), (4, 5)], [2, 4, 5], "hand"))


def test_size_beyond_the_scratch_is_refused(mc):
    import torch
    g = synth.config1()
    csr = mc.build_csr(g.n, g.src, g.dst, transposed=False)
    acc = torch.from_numpy(g.acc).to(csr.row_ptr.device)
    res = mc.new_result(csr.row_ptr.device)
    rc = mc.map_detect_noalloc(mc.MAP_NOALLOC_MAX_N + 1, csr.row_ptr, csr.col, acc, res, None, None, 0, 0)
    assert rc == mc.MAP_ERANGE
