"""Serving engine (one persistent launch that takes jobs while it runs): each
job's CSR equals map_build_csr's and its result equals the oracle's
(bit-exact), across gang sizes, slot reuse, bad input and the engine's own
exits.  No test synchronizes the whole device while an engine runs (the
engine stays resident until it is stopped)."""
import time

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


def _graphs():
    gs = [synth.config4(i) for i in range(0, 10)]
    gs += [synth.random_graph(700 + i, n, int(n * 1.5), p_acc=0.1) for i, n in enumerate([1, 2, 64, 129, 3000])]
    gs += [synth.config1(seed=8), synth.config1(seed=8, dag=True), synth.config2(seed=9, n=1 << 14, planted=True),
           synth.config2(seed=10, n=1 << 15, planted=False)]
    gs += [synth.from_edges(5, [(1, 2), (2, 3), (3, 1), (3, 4), (4, 5)], [2, 4, 5], "hand"),
           synth.from_edges(3, [], [], "empty-acc"), synth.from_edges(4, [], [1, 3], "no-edges")]
    return gs


class _Job:
    def __init__(self, mc, g, gang, host=False):
        import torch
        dev = torch.device("cuda")
        self.g, self.gang = g, gang
        m = g.m
        # edges and flags on the device, or left in pinned host memory for the engine to read over the bus
        put = (lambda a: torch.from_numpy(a).pin_memory()) if host else (lambda a: torch.from_numpy(a).to(dev))
        self.src = put(g.src) if m else None
        self.dst = put(g.dst) if m else None
        self.row_ptr = torch.full((g.n + 1,), -7, dtype=torch.int32, device=dev)
        self.col = torch.full((max(m, 1),), -7, dtype=torch.int32, device=dev)
        self.acc = put(g.acc)
        self.scratch = torch.empty(mc.map_job_scratch_bytes(g.n, m), dtype=torch.uint8, device=dev)
        self.ref_csr = mc.build_csr(g.n, g.src, g.dst, transposed=False) if m else None
        self.result = None


def _run(mc, eng, jobs, deadline_s=60.0):
    """Submit every job (retrying on a full engine) and poll them all to completion."""
    pending = list(jobs)
    running = {}
    t0 = time.perf_counter()
    while pending or running:
        while pending:
            j = pending[0]
            slot = eng.submit(j.g.n, j.src, j.dst, j.row_ptr, j.col, j.acc, j.scratch, gang=j.gang)
            if slot is None:
                break
            running[slot] = pending.pop(0)
        for slot in list(running):
            r = eng.poll(slot)
            if r is not None:
                running.pop(slot).result = r
        assert time.perf_counter() - t0 < deadline_s, "engine jobs did not finish"
        time.sleep(50e-6)


def _check(mc, jobs):
    for j in jobs:
        ref = oracle.map_detect(j.g, mode="desc")
        r = j.result
        assert r.status == 0, (j.g.name, j.gang, r)
        assert r.verdict == ref.verdict, (j.g.name, j.gang, r.verdict, ref.verdict)
        assert r.accepting_left == ref.accepting_left, (j.g.name, j.gang)
        if j.ref_csr is not None:
            rp = j.row_ptr.cpu().numpy()
            assert np.array_equal(rp, j.ref_csr.row_ptr.cpu().numpy()), j.g.name
            m = int(rp[-1])
            col, rcol = j.col.cpu().numpy()[:m], j.ref_csr.col.cpu().numpy()[:m]
            rows = np.repeat(np.arange(j.g.n), np.diff(rp))     # each row's columns as a multiset
            assert np.array_equal(col[np.lexsort((col, rows))], rcol[np.lexsort((rcol, rows))]), j.g.name


def test_engine_jobs_match_oracle_and_csr(mc):
    gs = _graphs()
    gangs = [1, 2, 3, 8, 16, 1, 4]
    jobs = [_Job(mc, g, gangs[i % len(gangs)], host=i % 2 == 1) for i, g in enumerate(gs)]
    jobs += [_Job(mc, gs[i], 64, host=True) for i in (0, 15)]  # wide gangs on small graphs
    import torch
    torch.cuda.synchronize()
    with mc.Engine(max_jobs=64, idle_seconds=30.0) as eng:
        assert eng.workgroups >= 64
        _run(mc, eng, jobs)
    _check(mc, jobs)


def test_engine_direction_jobs_match_oracle_and_csr(mc):
    """MAP_FLAG_DIRECTION: each job also builds its transposed CSR and runs
    filtered sweeps with push rounds on small frontiers; results exact."""
    gs = _graphs()
    gangs = [1, 2, 3, 8, 1, 4]
    jobs = [_Job(mc, g, gangs[i % len(gangs)], host=i % 2 == 0) for i, g in enumerate(gs)]
    import torch
    torch.cuda.synchronize()
    with mc.Engine(max_jobs=64, idle_seconds=30.0, flags=mc.MAP_FLAG_DIRECTION) as eng:
        _run(mc, eng, jobs)
    _check(mc, jobs)
    # The transposed CSR each job built in its scratch (after the packed values,
    # flags, four bitmaps, scan partials and the staged edge list, each part
    # 256-aligned) equals map_build_csr's, row by row as a multiset.
    al = lambda x: (x + 255) // 256 * 256
    for j in jobs:
        n, m = j.g.n, j.g.m
        if m == 0:
            continue
        ref = mc.build_csr(n, j.g.src, j.g.dst, transposed=True)
        off = al(4 * n) + al(n) + 4 * al((n + 31) // 32 * 4) + 256 * 4 + 2 * al(4 * m)
        sc = j.scratch.cpu().numpy()
        rp = sc[off:off + 4 * (n + 1)].view(np.int32)
        col = sc[off + al(4 * n + 4):off + al(4 * n + 4) + 4 * m].view(np.int32)
        assert np.array_equal(rp, ref.rrow_ptr.cpu().numpy()), j.g.name
        rcol = ref.rcol.cpu().numpy()
        rows = np.repeat(np.arange(n), np.diff(rp))
        assert np.array_equal(col[np.lexsort((col, rows))], rcol[np.lexsort((rcol, rows))]), j.g.name


def test_engine_slot_reuse_when_full(mc):
    gs = [synth.random_graph(900 + i, 200 + 37 * i, 600 + 50 * i, p_acc=0.2) for i in range(16)]
    jobs = [_Job(mc, g, 1 + i % 3) for i, g in enumerate(gs)]
    import torch
    torch.cuda.synchronize()
    with mc.Engine(max_jobs=3, idle_seconds=30.0) as eng:
        _run(mc, eng, jobs)
    _check(mc, jobs)


def test_engine_bad_edge_then_good_job(mc):
    import torch
    bad = synth.from_edges(4, [(1, 2), (2, 3)], [2], "bad")
    bad_dst = bad.dst.copy()
    bad_dst[1] = 5                                             # outside 1..4
    good = synth.config1(seed=21)
    jb = _Job(mc, bad, 2)
    jb.dst = torch.from_numpy(bad_dst).cuda()
    jg = _Job(mc, good, 4)
    torch.cuda.synchronize()
    with mc.Engine(max_jobs=8, idle_seconds=30.0) as eng:
        _run(mc, eng, [jb])
        _run(mc, eng, [jg])
    assert jb.result.status == mc.MAP_ERANGE_DEV
    assert jb.result.verdict == (0, 0, 0)
    _check(mc, [jg])


def test_engine_idle_bound_ends_the_kernel(mc):
    import torch
    g = synth.config1(seed=22)
    j = _Job(mc, g, 1)
    torch.cuda.synchronize()
    eng = mc.Engine(max_jobs=4, idle_seconds=0.3)
    try:
        time.sleep(1.5)
        with pytest.raises(mc.MapError) as e:
            eng.submit(g.n, j.src, j.dst, j.row_ptr, j.col, j.acc, j.scratch, gang=1)
        assert e.value.status == mc.MAP_EDEVICE
    finally:
        eng.close()
    torch.cuda.synchronize()


def test_engine_stop_without_jobs_and_after_stop(mc):
    import torch
    g = synth.config1(seed=23)
    j = _Job(mc, g, 1)
    torch.cuda.synchronize()
    eng = mc.Engine(max_jobs=4, idle_seconds=30.0)
    try:
        eng.stop()
        with pytest.raises(mc.MapError) as e:
            eng.submit(g.n, j.src, j.dst, j.row_ptr, j.col, j.acc, j.scratch, gang=1)
        assert e.value.status == mc.MAP_EINVAL
    finally:
        eng.close()
    torch.cuda.synchronize()
    with mc.Engine(max_jobs=4, idle_seconds=30.0):
        pass
    torch.cuda.synchronize()


def test_engine_rejects_pageable_and_host_outputs(mc):
    import torch
    g = synth.config1(seed=24)
    j = _Job(mc, g, 1)
    page_src = torch.from_numpy(g.src.copy())                  # pageable: the device cannot read it
    host_rp = torch.empty(g.n + 1, dtype=torch.int32).pin_memory()
    torch.cuda.synchronize()
    with mc.Engine(max_jobs=4, idle_seconds=30.0) as eng:
        for args in ((page_src, j.dst, j.row_ptr, j.acc), (j.src, j.dst, host_rp, j.acc),
                     (j.src, j.dst, j.row_ptr, torch.from_numpy(g.acc.copy()))):
            src, dst, rp, acc = args
            with pytest.raises(mc.MapError) as e:
                eng.submit(g.n, src, dst, rp, j.col, acc, j.scratch, gang=1)
            assert e.value.status == mc.MAP_EINVAL
        _run(mc, eng, [j])                                      # the engine still serves valid jobs
    _check(mc, [j])


def test_engine_concurrent_gangs_in_adjacent_slots(mc):
    """Many multi-workgroup jobs at once through few job slots: a job's set-up
    (clearing its slot's control blocks) runs while the jobs in neighbouring
    slots are inside their barriers, and must not disturb them."""
    import torch
    gs = [synth.config4(i) for i in range(40, 76)]
    jobs = [_Job(mc, g, 4 + (i % 5) * 7, host=i % 3 == 0) for i, g in enumerate(gs)]
    torch.cuda.synchronize()
    with mc.Engine(max_jobs=6, idle_seconds=30.0) as eng:
        _run(mc, eng, jobs)
        _run(mc, eng, jobs[:12])                                # slots reused by a second wave
    _check(mc, jobs)
