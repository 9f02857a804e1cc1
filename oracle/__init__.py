"""CPU oracle for MAP accepting-cycle detection -- test infrastructure only.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
use this package.  The product path (the HIP library and its binding) never
imports, links or calls it, and the two share no code.

The arithmetic lives in ``map_oracle.c`` (plain C, compiled with gcc by
``build()``); this module marshals numpy arrays.  See the C file's header for
the method as the paper states it (Section 2) and the readings taken where it
is silent.

Functions
---------
fixpoint(g, acc, mode)  map vector of one fixpoint; mode 'jacobi' (the value
                        propagation as stated), 'reach' (definition, tiny
                        graphs) or 'desc' (definition by decreasing accepting
                        id, O(n+m))
map_detect(g, ...)      the MAP outer loop: found, witness, K, trace, maps
digest(map)             order-independent 64-bit digest of a map vector
jacobi_steps(g, acc)    the vector after every jacobi pass
tarjan(g)               accepting-cycle verdict from strongly connected components
ndfs(g)                 accepting-cycle verdict from nested depth-first search
lasso(g, w, init)       counterexample: shortest path init -> w, then shortest
                        cycle through w (breadth-first search over successors)
trim(g)                 relevance pruning: vertices left after repeatedly
                        removing those with no remaining predecessor or
                        successor, and the accepting flags restricted to them
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")
_SRC = os.path.join(_HERE, "map_oracle.c")
MODES = {"jacobi": 0, "reach": 1, "desc": 2}
_BASE_FLAGS = ["-O2", "-std=gnu11", "-fPIC", "-shared", "-Wall"]
# Build flavours of the same source: the plain single-threaded oracle, and the
# OpenMP one (the jacobi pass's edge loop shared among the host's threads),
# used only to time the jacobi route on all host cores.
_FLAVOURS = {_LIB_PATH: [], _OMP_PATH: ["-fopenmp", "-DORACLE_OPENMP"]}


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` (single-threaded C) and ``liboracle_omp.so`` next to this file with gcc."""
    for path, extra in _FLAVOURS.items():
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            subprocess.check_call(["gcc", *_BASE_FLAGS, *extra, "-o", tmp, _SRC])
            os.replace(tmp, path)
    return _LIB_PATH


def build_sanitized(out_dir: str) -> str:
    """The plain oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
    (host code only), for running the pins under the sanitizers."""
    path = os.path.join(out_dir, "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=gnu11", "-fPIC", "-shared", "-Wall",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           "-o", path, _SRC])
    return path


_lib = None
_libs = {}
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")


def _load(omp: bool = False):
    global _lib
    path = _OMP_PATH if omp else os.environ.get("ORACLE_LIB", _LIB_PATH)
    if path not in _libs:
        if not os.path.exists(path):
            build(force=False)
        lib = ctypes.CDLL(path)
        i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        lib.oracle_fixpoint.argtypes = [i32, i64, _i32p, _i32p, _u8p, i32, _i32p, ctypes.POINTER(i64)]
        lib.oracle_fixpoint.restype = ctypes.c_int
        lib.oracle_digest.argtypes = [i32, _i32p]
        lib.oracle_digest.restype = ctypes.c_uint64
        lib.oracle_map_detect.argtypes = [i32, i64, _i32p, _i32p, _u8p, i32, i32, _i32p, ctypes.POINTER(i64),
                                          vp, i32, vp, i32, vp]
        lib.oracle_map_detect.restype = ctypes.c_int
        lib.oracle_tarjan.argtypes = [i32, i64, _i32p, _i32p, _u8p, vp]
        lib.oracle_tarjan.restype = ctypes.c_int
        lib.oracle_ndfs.argtypes = [i32, i64, _i32p, _i32p, _u8p]
        lib.oracle_ndfs.restype = ctypes.c_int
        lib.oracle_jacobi_steps.argtypes = [i32, i64, _i32p, _i32p, _u8p, vp, i64]
        lib.oracle_jacobi_steps.restype = i64
        lib.oracle_lasso.argtypes = [i32, i64, _i32p, _i32p, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                     vp, i32]
        lib.oracle_lasso.restype = ctypes.c_int
        lib.oracle_trim.argtypes = [i32, i64, _i32p, _i32p, _u8p, _u8p, _u8p]
        lib.oracle_trim.restype = i64
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = ctypes.c_int
        _libs[path] = lib
        if not omp:
            _lib = lib
    return _libs[path]


def threads(omp: bool = False) -> int:
    """Host threads the jacobi route uses in the plain (1) or OpenMP build."""
    return int(_load(omp).oracle_threads())


def _arrays(g, acc=None):
    src = np.ascontiguousarray(g.src, dtype=np.int32)
    dst = np.ascontiguousarray(g.dst, dtype=np.int32)
    a = np.ascontiguousarray(g.acc if acc is None else acc, dtype=np.uint8)
    if a.shape != (g.n,):
        raise ValueError("accepting vector must have n entries")
    return src, dst, a


def fixpoint(g, acc=None, mode: str = "jacobi"):
    """Return (map vector int32[n], sweeps) for accepting set ``acc`` (default g.acc)."""
    src, dst, a = _arrays(g, acc)
    out = np.zeros(g.n, np.int32)
    sweeps = ctypes.c_int64(0)
    rc = _load().oracle_fixpoint(g.n, len(src), src, dst, a, MODES[mode], out, ctypes.byref(sweeps))
    if rc != 0:
        raise ValueError(f"oracle_fixpoint failed rc={rc}")
    return out, int(sweeps.value)


def jacobi_steps(g, acc=None, cap: int = 1 << 16) -> np.ndarray:
    """The vectors after each jacobi pass (the last pass changes nothing)."""
    src, dst, a = _arrays(g, acc)
    buf = np.zeros((cap, g.n), np.int32)
    t = int(_load().oracle_jacobi_steps(g.n, len(src), src, dst, a, buf.ctypes.data, cap))
    if t < 0:
        raise ValueError(f"oracle_jacobi_steps failed rc={t}")
    return buf[:min(t, cap)].copy()


def digest(map_vec) -> int:
    m = np.ascontiguousarray(map_vec, dtype=np.int32)
    return int(_load().oracle_digest(len(m), m))


@dataclass
class Detect:
    found: int
    witness: int
    iterations: int
    accepting_left: int
    sweeps: int
    status: int
    trace: np.ndarray      # uint64 [K_recorded, 3]: |Del_k|, sweeps_k, digest_k
    maps: np.ndarray       # int32 [min(K, maps_cap), n]
    acc_out: np.ndarray    # uint8 [n]

    @property
    def verdict(self):
        return (self.found, self.witness, self.iterations)


def map_detect(g, acc=None, mode: str = "desc", max_iterations: int = 0, trace_cap: int | None = None,
               maps_cap: int = 0, omp: bool = False) -> Detect:
    """Run the MAP outer loop on the oracle (``omp``: the OpenMP build, same results)."""
    src, dst, a = _arrays(g, acc)
    n = g.n
    if trace_cap is None:
        trace_cap = int(a.sum()) + 1
    trace = np.zeros((max(trace_cap, 1), 3), np.uint64)
    maps = np.zeros((max(maps_cap, 0), n), np.int32)
    acc_out = np.zeros(n, np.uint8)
    res = np.zeros(4, np.int32)
    sweeps = ctypes.c_int64(0)
    rc = _load(omp).oracle_map_detect(n, len(src), src, dst, a, MODES[mode], max_iterations, res,
                                   ctypes.byref(sweeps), trace.ctypes.data, trace_cap,
                                   maps.ctypes.data if maps_cap > 0 else None, maps_cap,
                                   acc_out.ctypes.data)
    if rc not in (0, -5):
        raise ValueError(f"oracle_map_detect failed rc={rc}")
    k = int(res[2])
    return Detect(found=int(res[0]), witness=int(res[1]), iterations=k, accepting_left=int(res[3]),
                  sweeps=int(sweeps.value), status=rc, trace=trace[:min(k, trace_cap)].copy(),
                  maps=maps[:min(k, maps_cap)].copy(), acc_out=acc_out)


def tarjan(g, acc=None, with_components: bool = False):
    src, dst, a = _arrays(g, acc)
    comp = np.zeros(g.n, np.int32)
    rc = _load().oracle_tarjan(g.n, len(src), src, dst, a, comp.ctypes.data)
    if rc < 0:
        raise ValueError(f"oracle_tarjan failed rc={rc}")
    return (rc, comp) if with_components else rc


def ndfs(g, acc=None) -> int:
    src, dst, a = _arrays(g, acc)
    rc = _load().oracle_ndfs(g.n, len(src), src, dst, a)
    if rc < 0:
        raise ValueError(f"oracle_ndfs failed rc={rc}")
    return rc


@dataclass
class Lasso:
    status: str              # "ok", "no_path" (init does not reach w, or w on no cycle), "no_space"
    stem_len: int            # edges init -> w (0 without init); -1 if not found
    cycle_len: int           # edges of a shortest cycle through w; -1 if none
    path: np.ndarray | None  # int32 ids: init, ..., w, ..., w (stem_len + cycle_len + 1), or None


def lasso(g, w: int, init: int = 0, cap: int | None = None) -> Lasso:
    """Counterexample for witness ``w``: shortest stem from ``init`` (0: none), shortest cycle through w."""
    src, dst, _ = _arrays(g, np.zeros(g.n, np.uint8))
    cap = g.n + g.n + 1 if cap is None else cap
    path = np.zeros(max(cap, 1), np.int32)
    s_len, c_len = ctypes.c_int32(0), ctypes.c_int32(0)
    rc = _load().oracle_lasso(g.n, len(src), src, dst, int(w), int(init), ctypes.byref(s_len), ctypes.byref(c_len),
                              path.ctypes.data, cap)
    if rc not in (0, -8, -9):
        raise ValueError(f"oracle_lasso failed rc={rc}")
    status = {0: "ok", -8: "no_path", -9: "no_space"}[rc]
    s, c = int(s_len.value), int(c_len.value)
    return Lasso(status, s, c, path[:s + c + 1].copy() if rc == 0 else None)


def trim(g, acc=None):
    """(keep uint8[n], accepting flags & keep) after trimming cycle-free vertices."""
    src, dst, a = _arrays(g, acc)
    keep = np.zeros(g.n, np.uint8)
    acc_out = np.zeros(g.n, np.uint8)
    k = int(_load().oracle_trim(g.n, len(src), src, dst, a, keep, acc_out))
    if k < 0:
        raise ValueError(f"oracle_trim failed rc={k}")
    return keep, acc_out
