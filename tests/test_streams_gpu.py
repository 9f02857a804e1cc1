"""Calls on side streams, and on two streams at once, through the C ABI.

The convenience wrappers take a ``stream`` and must upload, call and read back
on it: a result read on torch's current stream while the call still runs on
the side stream would be the zeroed result buffer.  The header also allows
calls on different streams with disjoint outputs and workspaces to run
concurrently.  Every result is compared with the oracle's.
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


def test_wrappers_on_a_side_stream(mc):
    import torch
    g = synth.config2(seed=3, n=1 << 15, planted=True)
    say("side stream", g.name, "n", g.n, "m", len(g.src))
    ref = oracle.map_detect(g)
    assert ref.found == 1
    s = torch.cuda.Stream()
    csr = mc.build_csr(g.n, g.src, g.dst, transposed=True, stream=s)
    out = mc.detect(csr, g.acc, want_acc=True, stream=s)
    assert out.result.status == 0
    assert out.result.verdict == ref.verdict
    assert out.result.accepting_left == ref.accepting_left
    assert np.array_equal(out.accepting_out, ref.acc_out)

    got, res = mc.propagate(csr, g.acc, stream=s)
    want, _ = oracle.fixpoint(g)
    assert res.status == 0
    with torch.cuda.stream(s):
        assert np.array_equal(got.cpu().numpy(), want)

    t = mc.trim(csr, g.acc, stream=s)
    keep, acc = oracle.trim(g)
    assert t.status == mc.MAP_OK and (t.kept, t.accepting_kept) == (int(keep.sum()), int(acc.sum()))

    w = ref.witness
    lo = mc.lasso(csr, w, 1, stream=s)
    lw = oracle.lasso(g, w, 1)
    assert lw.status == "ok" and lo.status == mc.MAP_OK
    assert (lo.stem_len, lo.cycle_len) == (lw.stem_len, lw.cycle_len)
    say("  verdict", out.result.verdict, "lasso", lo.stem_len, lo.cycle_len)


def test_two_streams_at_once(mc):
    """Three graphs on two streams, enqueued back to back with no wait between them."""
    import torch
    graphs = [synth.config2(seed=3, n=1 << 15, planted=True), synth.config2(seed=7, n=1 << 16), synth.config1()]
    refs = [oracle.map_detect(g) for g in graphs]
    jobs = []
    for g in graphs:
        csr = mc.build_csr(g.n, g.src, g.dst, transposed=False)
        acc = torch.as_tensor(g.acc, dtype=torch.uint8).cuda()
        res = mc.new_result()
        acc_out = torch.zeros(g.n, dtype=torch.uint8, device="cuda")
        ws = mc.workspace(g.n, len(g.src))
        jobs.append((g, csr, acc, res, acc_out, ws))
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for i, (g, csr, acc, res, acc_out, ws) in enumerate(jobs):
        say("two streams: enqueue", g.name, "n", g.n, "on stream", 1 + i % 2)
        rc = mc.map_detect(g.n, csr.row_ptr, csr.col, None, None, acc, res, None, acc_out, 0, 0, ws,
                           s1 if i % 2 == 0 else s2)
        assert rc == mc.MAP_OK
    s1.synchronize()
    s2.synchronize()
    for (g, csr, acc, res, acc_out, ws), ref in zip(jobs, refs):
        r = mc.Result.from_tensor(res)
        say("  ", g.name, "verdict", r.verdict, "oracle", ref.verdict, "status", r.status)
        assert r.status == 0
        assert r.verdict == ref.verdict
        assert r.accepting_left == ref.accepting_left
        assert np.array_equal(acc_out.cpu().numpy(), ref.acc_out)


def test_two_host_threads(mc):
    """Two host threads, each on its own stream, build and detect at the same
    time (the binding releases the interpreter lock during library calls)."""
    import threading

    import torch
    graphs = [synth.config2(seed=5, n=1 << 16, planted=True), synth.config2(seed=9, n=1 << 15)]
    refs = [oracle.map_detect(g) for g in graphs]
    out = [None, None]
    errors = []

    def work(i):
        try:
            torch.cuda.set_device(0)
            s = torch.cuda.Stream()
            g = graphs[i]
            csr = mc.build_csr(g.n, g.src, g.dst, transposed=False, stream=s)
            out[i] = mc.detect(csr, g.acc, want_acc=True, stream=s)
        except Exception as e:  # reported below, in the test's own thread
            errors.append(repr(e))

    threads = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=100)
    assert not any(t.is_alive() for t in threads), "a worker thread did not finish"
    assert not errors, errors
    for g, o, ref in zip(graphs, out, refs):
        say("  thread", g.name, "verdict", o.result.verdict, "oracle", ref.verdict)
        assert o.result.status == 0
        assert o.result.verdict == ref.verdict
        assert np.array_equal(o.accepting_out, ref.acc_out)
