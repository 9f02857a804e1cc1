"""Seeded synthetic inputs for MAP accepting-cycle detection.

Input generation only: this module holds none of the method's arithmetic.  The
CPU oracle and the HIP library both consume the numpy arrays returned here, so
the two sides always see identical inputs.

Each generator returns a ``Graph``: ``n`` vertices with ids 1..n, an edge list
``src -> dst`` of the generated state graph G (int32, 1-based), and
``acc`` (uint8[n], ``acc[i]`` flags id ``i+1`` as accepting).

Workload shapes (the paper's DVE models are not available; these stand in for
state spaces that are BFS-numbered and forward-heavy with loop-closing back
edges):

========  =====================================================================
config 1  n=10,000, out-degree U{1..4}, targets U[1,n], 5% accepting;
          ``dag=True`` keeps only high->low edges of the same draw
config 2  n=2**20 in BFS order, out-degree 1+Poisson(3), 80% local (offset
          <=1024) / 20% uniform, 90% forward / 10% back, 1% accepting; back
          edges never span an accepting id (variant B: no accepting cycle);
          ``planted=True`` adds one accepting 64-cycle (variant A)
config 3  n=2**25 DAG, vertex v>=2 has U{1..7} edges to U[1,v-1], 0.1%
          accepting
config 4  graph ``index`` of a batch: log-uniform n in [1e3,1e6], config-1
          draw in DAG form, 5% accepting, odd indices planted
config 5  query ``index`` of a serving stream: log-uniform n in [1e4,4e6],
          accepting ratio U[0.1%,5%], config-4 recipe
========  =====================================================================
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_SRC = os.path.join(_HERE, "gen.c")


def build(force: bool = True) -> str:
    """Compile ``libsynth.so`` next to this file with gcc."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _SynthGraph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64),
                ("src", ctypes.POINTER(ctypes.c_int32)), ("dst", ctypes.POINTER(ctypes.c_int32)),
                ("acc", ctypes.POINTER(ctypes.c_uint8)), ("n_acc", ctypes.c_int32),
                ("n_planted", ctypes.c_int32), ("planted", ctypes.c_int32 * 64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(_SynthGraph)
        u64, i32 = ctypes.c_uint64, ctypes.c_int32
        lib.synth_config1.argtypes = [u64, i32, ctypes.c_int, P]
        lib.synth_config2.argtypes = [u64, i32, ctypes.c_int, P]
        lib.synth_config3.argtypes = [u64, i32, P]
        lib.synth_config4.argtypes = [u64, i32, P]
        lib.synth_config5.argtypes = [u64, i32, P]
        lib.synth_config4_n.argtypes = [u64, i32]
        lib.synth_config4_n.restype = i32
        lib.synth_config5_meta.argtypes = [u64, i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double)]
        lib.synth_free.argtypes = [P]
        for f in (lib.synth_config1, lib.synth_config2, lib.synth_config3, lib.synth_config4,
                  lib.synth_config5, lib.synth_config5_meta):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class Graph:
    """A generated graph: ids 1..n, edges src->dst of G, accepting flags."""
    n: int
    src: np.ndarray
    dst: np.ndarray
    acc: np.ndarray
    name: str = ""
    planted: list = field(default_factory=list)

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    @property
    def n_acc(self) -> int:
        return int(self.acc.sum())


def _take(g: _SynthGraph, name: str) -> Graph:
    n, m = int(g.n), int(g.m)
    src = np.ctypeslib.as_array(g.src, shape=(m,)).copy() if m else np.zeros(0, np.int32)
    dst = np.ctypeslib.as_array(g.dst, shape=(m,)).copy() if m else np.zeros(0, np.int32)
    acc = np.ctypeslib.as_array(g.acc, shape=(n,)).copy()
    planted = [int(g.planted[i]) for i in range(g.n_planted)]
    _load().synth_free(ctypes.byref(g))
    return Graph(n=n, src=src, dst=dst, acc=acc, name=name, planted=planted)


def _call(fn, name, *args) -> Graph:
    g = _SynthGraph()
    rc = fn(*args, ctypes.byref(g))
    if rc != 0:
        raise RuntimeError(f"generator {name} failed (rc={rc})")
    return _take(g, name)


def config1(seed: int = 1, n: int = 10_000, dag: bool = False) -> Graph:
    return _call(_load().synth_config1, f"c1{'b' if dag else 'a'}(n={n},seed={seed})", seed, n, int(dag))


def config2(seed: int = 2, n: int = 1 << 20, planted: bool = False) -> Graph:
    return _call(_load().synth_config2, f"c2{'A' if planted else 'B'}(n={n},seed={seed})", seed, n,
                 int(planted))


def config3(seed: int = 3, n: int = 1 << 25) -> Graph:
    return _call(_load().synth_config3, f"c3(n={n},seed={seed})", seed, n)


def config4(index: int, seed: int = 4) -> Graph:
    return _call(_load().synth_config4, f"c4[{index}](seed={seed})", seed, index)


def config4_n(index: int, seed: int = 4) -> int:
    return int(_load().synth_config4_n(seed, index))


def config5_meta(index: int, seed: int = 5):
    """(n, accepting ratio, unit-mean exponential inter-arrival gap) of query ``index``."""
    n = ctypes.c_int32()
    ratio = ctypes.c_double()
    gap = ctypes.c_double()
    _load().synth_config5_meta(seed, index, ctypes.byref(n), ctypes.byref(ratio), ctypes.byref(gap))
    return int(n.value), float(ratio.value), float(gap.value)


def config5(index: int, seed: int = 5) -> Graph:
    return _call(_load().synth_config5, f"c5[{index}](seed={seed})", seed, index)


def from_edges(n: int, edges, accepting, name: str = "") -> Graph:
    """Build a Graph from python edge pairs (1-based) and accepting ids."""
    e = np.asarray(list(edges), dtype=np.int32).reshape(-1, 2)
    acc = np.zeros(n, np.uint8)
    for a in accepting:
        acc[int(a) - 1] = 1
    return Graph(n=n, src=e[:, 0].copy(), dst=e[:, 1].copy(), acc=acc, name=name)


def random_graph(seed: int, n: int, m: int, p_acc: float = 0.2, self_loops: bool = True) -> Graph:
    """Small uniform random graph for property tests (numpy's seeded generator)."""
    rng = np.random.default_rng(seed)
    src = rng.integers(1, n + 1, size=m, dtype=np.int64).astype(np.int32)
    dst = rng.integers(1, n + 1, size=m, dtype=np.int64).astype(np.int32)
    if not self_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    acc = (rng.random(n) < p_acc).astype(np.uint8)
    return Graph(n=n, src=src, dst=dst, acc=acc, name=f"rand(n={n},m={m},seed={seed})")


def generation_order(g: Graph) -> Graph:
    """The same graph with its edges in the order a breadth-first state generator emits them: grouped by
    source id, ascending (stable within a source).  Generated edge lists are already grouped that way except
    for edges appended afterwards (the planted cycle), which this moves to their source's place."""
    order = np.argsort(g.src, kind="stable")
    return Graph(n=g.n, src=g.src[order].copy(), dst=g.dst[order].copy(), acc=g.acc.copy(),
                 name=g.name + "/gen-order", planted=list(g.planted))


def prefix(g: Graph, m: int) -> Graph:
    """The graph of the first m edges (all n vertices, same accepting flags)."""
    return Graph(n=g.n, src=g.src[:m].copy(), dst=g.dst[:m].copy(), acc=g.acc.copy(), name=f"{g.name}[:{m}]")
