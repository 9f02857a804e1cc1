"""MI355X-native MAP accepting-cycle detection (Barnat, Brim, Ceska, PDMC 2009).

Thin Python binding over the C ABI of ``libmapcheck.so`` (declared in
``include/mapcheck.h``).  Every step of the method runs in the library's HIP
kernels; this module only marshals arguments.  PyTorch supplies device memory
(CUDA tensors on ROCm) and the current stream.

The raw calls mirror the C names and never synchronize:

``map_workspace_bytes(n, m, flags)``
``map_build_csr(n, src, dst, row_ptr, col, rrow_ptr, rcol, status, ws)``
``map_propagate(n, row_ptr, col, rrow_ptr, rcol, accepting, map_out, result, flags, ws)``
``map_detect(n, row_ptr, col, rrow_ptr, rcol, accepting0, result, trace, accepting_out, max_iterations, flags, ws)``
``map_lasso(n, row_ptr, col, witness, init, path, result, ws)``
``map_trim(n, row_ptr, col, rrow_ptr, rcol, accepting, keep_out, accepting_out, result, ws)``

Convenience wrappers (``Csr``, ``build_csr``, ``propagate``, ``detect``, ``lasso``, ``trim``)
allocate the tensors, call the raw entry points and synchronize when results
are read back.

The library must be built (``python paper_0912_2555_amd/build.py``); importing
this package raises if ``libmapcheck.so`` is missing -- there is no fallback.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
# MAPCHECK_LIB may name the phase-clock measurement build of the same source
# (libmapcheck_phases.so); either way a missing library is an import error.
LIB_PATH = os.environ.get("MAPCHECK_LIB") or os.path.join(_PKG, "libmapcheck.so")

MAP_OK = 0
MAP_EINVAL = -1
MAP_ERANGE = -2
MAP_ENOSPC = -3
MAP_EDEVICE = -4
MAP_ENOTCONVERGED = -5
MAP_ERANGE_DEV = -6
MAP_EBUSY = -7
MAP_ENOPATH = -8
MAP_PENDING = 1
MAP_FLAG_DENSE_ONLY = 0x1
MAP_FLAG_NO_TRACE_DIGEST = 0x2
MAP_FLAG_STREAM = 0x4
MAP_FLAG_SYNC_SWEEPS = 0x8
MAP_FLAG_PUSH = 0x10
MAP_FLAG_EARLY = 0x20
MAP_FLAG_NO_FILTER = 0x40
MAP_FLAG_DIRECTION = 0x80
MAP_NOALLOC_MAX_N = 1 << 22

EXPORTS = ("map_workspace_bytes", "map_build_csr", "map_propagate", "map_detect", "map_batch_workspace_bytes",
           "map_detect_batch", "map_job_scratch_bytes", "map_engine_create", "map_engine_workgroups",
           "map_engine_submit", "map_engine_poll", "map_engine_stop", "map_engine_destroy", "map_lasso",
           "map_trim", "map_strerror", "map_detect_noalloc", "map_phase_counters")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_0912_2555_amd/build.py` "
                      "(there is no fallback implementation)")

_lib = ctypes.CDLL(LIB_PATH)
_vp, _i32, _i64, _u32, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t
_lib.map_workspace_bytes.argtypes = [_i32, _i64, _u32]
_lib.map_workspace_bytes.restype = _sz
_lib.map_build_csr.argtypes = [_i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
_lib.map_build_csr.restype = ctypes.c_int
_lib.map_propagate.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _u32, _vp, _sz, _vp]
_lib.map_propagate.restype = ctypes.c_int
_lib.map_detect.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _i32, _u32, _vp, _sz, _vp]
_lib.map_detect.restype = ctypes.c_int
_lib.map_detect_noalloc.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _i32, _u32, _vp]
_lib.map_detect_noalloc.restype = ctypes.c_int
_lib.map_lasso.argtypes = [_i32, _vp, _vp, _i32, _i32, _vp, _i32, _vp, _vp, _sz, _vp]
_lib.map_lasso.restype = ctypes.c_int
_lib.map_trim.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
_lib.map_trim.restype = ctypes.c_int
_lib.map_batch_workspace_bytes.argtypes = [_i32, _i64, _u32]
_lib.map_batch_workspace_bytes.restype = _sz
_lib.map_detect_batch.argtypes = [_i32, _vp, _vp, _vp, _i64, _u32, _vp, _sz, _vp]
_lib.map_detect_batch.restype = ctypes.c_int
_lib.map_job_scratch_bytes.argtypes = [_i32, _i64]
_lib.map_job_scratch_bytes.restype = _sz
_lib.map_engine_create.argtypes = [_i32, _i32, ctypes.c_double, _u32, _vp, ctypes.POINTER(_vp)]
_lib.map_engine_create.restype = ctypes.c_int
_lib.map_engine_workgroups.argtypes = [_vp]
_lib.map_engine_workgroups.restype = ctypes.c_int
_lib.map_engine_submit.argtypes = [_vp, _vp, ctypes.POINTER(_i32)]
_lib.map_engine_submit.restype = ctypes.c_int
_lib.map_engine_poll.argtypes = [_vp, _i32, _vp]
_lib.map_engine_poll.restype = ctypes.c_int
_lib.map_engine_stop.argtypes = [_vp]
_lib.map_engine_stop.restype = ctypes.c_int
_lib.map_engine_destroy.argtypes = [_vp]
_lib.map_engine_destroy.restype = ctypes.c_int
_lib.map_phase_counters.argtypes = [_vp, _i32, _vp]
_lib.map_phase_counters.restype = ctypes.c_int
_lib.map_strerror.argtypes = [ctypes.c_int]
_lib.map_strerror.restype = ctypes.c_char_p


class MapError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {strerror(status)} ({status})")
        self.status = status


def strerror(status: int) -> str:
    return _lib.map_strerror(int(status)).decode()


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch.Tensor or None")
    if not t.is_cuda:
        raise ValueError("device tensor required (torch CUDA/HIP tensor)")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor required")
    return ctypes.c_void_p(t.data_ptr())


def _addr(t):
    """Address of a contiguous tensor on the device or in host memory (the callee validates it)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch.Tensor or None")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor required")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _on(stream):
    """Context in which a convenience wrapper allocates, uploads, calls and reads
    back: ``stream`` when given, so that every step is ordered with the call,
    else torch's current stream."""
    return torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()


def _check(rc: int, where: str):
    if rc != MAP_OK:
        raise MapError(rc, where)


# ------------------------------------------------------------ raw C-ABI calls

def map_workspace_bytes(n: int, m: int, flags: int = 0) -> int:
    return int(_lib.map_workspace_bytes(n, m, flags))


def map_build_csr(n, src, dst, row_ptr, col, rrow_ptr, rcol, status, ws, stream=None) -> int:
    m = 0 if src is None else int(src.numel())
    return _lib.map_build_csr(n, m, _ptr(src), _ptr(dst), _ptr(row_ptr), _ptr(col), _ptr(rrow_ptr), _ptr(rcol),
                              _ptr(status), _ptr(ws), 0 if ws is None else ws.numel() * ws.element_size(),
                              _stream(stream))


def map_propagate(n, row_ptr, col, rrow_ptr, rcol, accepting, map_out, result, flags, ws, stream=None) -> int:
    return _lib.map_propagate(n, _ptr(row_ptr), _ptr(col), _ptr(rrow_ptr), _ptr(rcol), _ptr(accepting),
                              _ptr(map_out), _ptr(result), flags, _ptr(ws),
                              0 if ws is None else ws.numel() * ws.element_size(), _stream(stream))


def map_detect(n, row_ptr, col, rrow_ptr, rcol, accepting0, result, trace, accepting_out, max_iterations, flags,
               ws, stream=None) -> int:
    cap = 0 if trace is None else int(trace.shape[0])
    return _lib.map_detect(n, _ptr(row_ptr), _ptr(col), _ptr(rrow_ptr), _ptr(rcol), _ptr(accepting0),
                           _ptr(result), _ptr(trace), cap, _ptr(accepting_out), max_iterations, flags, _ptr(ws),
                           0 if ws is None else ws.numel() * ws.element_size(), _stream(stream))


def map_detect_noalloc(n, row_ptr, col, accepting0, result, trace, accepting_out, max_iterations, flags,
                       stream=None) -> int:
    cap = 0 if trace is None else int(trace.shape[0])
    return _lib.map_detect_noalloc(n, _ptr(row_ptr), _ptr(col), _ptr(accepting0), _ptr(result), _ptr(trace), cap,
                                   _ptr(accepting_out), max_iterations, flags, _stream(stream))


def phase_counters(max_blocks: int = 2048) -> np.ndarray:
    """Phase clocks of the last loop-kernel launch (measurement build only):
    uint64[workgroups, 16], columns as map_phase_counters documents."""
    out = np.zeros((max_blocks, 16), dtype=np.uint64)
    nb = ctypes.c_int32(0)
    _check(_lib.map_phase_counters(out.ctypes.data, max_blocks, ctypes.byref(nb)), "map_phase_counters")
    return out[:min(nb.value, max_blocks)].copy()


def map_lasso(n, row_ptr, col, witness, init, path, result, ws, stream=None) -> int:
    cap = 0 if path is None else int(path.numel())
    return _lib.map_lasso(n, _ptr(row_ptr), _ptr(col), witness, init, _ptr(path), cap, _ptr(result), _ptr(ws),
                          0 if ws is None else ws.numel() * ws.element_size(), _stream(stream))


def map_trim(n, row_ptr, col, rrow_ptr, rcol, accepting, keep_out, accepting_out, result, ws, stream=None) -> int:
    return _lib.map_trim(n, _ptr(row_ptr), _ptr(col), _ptr(rrow_ptr), _ptr(rcol), _ptr(accepting), _ptr(keep_out),
                         _ptr(accepting_out), _ptr(result), _ptr(ws),
                         0 if ws is None else ws.numel() * ws.element_size(), _stream(stream))


def map_batch_workspace_bytes(count: int, total_n: int, flags: int = 0) -> int:
    return int(_lib.map_batch_workspace_bytes(count, total_n, flags))


def map_detect_batch(count, graphs, gang, results, total_n, flags, ws, stream=None) -> int:
    return _lib.map_detect_batch(count, _ptr(graphs), _ptr(gang), _ptr(results), total_n, flags, _ptr(ws),
                                 0 if ws is None else ws.numel() * ws.element_size(), _stream(stream))


# ---------------------------------------------------------------- wrappers

@dataclass
class Result:
    found: int
    witness: int
    iterations: int
    status: int
    sweeps: int
    accepting_left: int

    @property
    def verdict(self):
        return (self.found, self.witness, self.iterations)

    @staticmethod
    def from_tensor(t: torch.Tensor) -> "Result":
        a = t.detach().cpu().numpy().view(np.int32)
        sweeps = int(a[4:6].view(np.int64)[0])
        return Result(int(a[0]), int(a[1]), int(a[2]), int(a[3]), sweeps, int(a[6]))


def new_result(device=None) -> torch.Tensor:
    """A zeroed device map_result (32 bytes, viewed as int32[8])."""
    return torch.zeros(8, dtype=torch.int32, device=device or "cuda")


def workspace(n: int, m: int, flags: int = 0, device=None) -> torch.Tensor:
    nbytes = map_workspace_bytes(n, m, flags)
    if nbytes == 0:
        raise MapError(MAP_ERANGE, "map_workspace_bytes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device or "cuda")


@dataclass
class Csr:
    """Pull CSR of G (row v = successors) and, optionally, the transposed CSR."""
    n: int
    m: int
    row_ptr: torch.Tensor
    col: torch.Tensor
    rrow_ptr: torch.Tensor | None
    rcol: torch.Tensor | None
    status: torch.Tensor


def build_csr(n: int, src, dst, transposed: bool = True, ws: torch.Tensor | None = None, stream=None,
              device="cuda") -> Csr:
    """Upload (if needed) the 1-based edge list and build the CSR on the device.

    With ``stream`` every step runs on it; the CSR is ready once it has run."""
    with _on(stream):
        src = torch.as_tensor(src, dtype=torch.int32).to(device).contiguous()
        dst = torch.as_tensor(dst, dtype=torch.int32).to(device).contiguous()
        m = int(src.numel())
        row_ptr = torch.empty(n + 1, dtype=torch.int32, device=device)
        col = torch.empty(max(m, 1), dtype=torch.int32, device=device)
        rrow_ptr = torch.empty(n + 1, dtype=torch.int32, device=device) if transposed else None
        rcol = torch.empty(max(m, 1), dtype=torch.int32, device=device) if transposed else None
        status = torch.zeros(1, dtype=torch.int32, device=device)
        if ws is None:
            ws = workspace(n, m, device=device)
        _check(map_build_csr(n, src if m else None, dst if m else None, row_ptr, col, rrow_ptr, rcol, status, ws,
                             stream), "map_build_csr")
    return Csr(n, m, row_ptr, col, rrow_ptr, rcol, status)


def propagate(csr: Csr, accepting, flags: int = 0, ws=None, stream=None):
    """One fixpoint: returns (map vector as a device int32 tensor, Result)."""
    with _on(stream):
        acc = torch.as_tensor(accepting, dtype=torch.uint8).to(csr.row_ptr.device).contiguous()
        out = torch.empty(csr.n, dtype=torch.int32, device=csr.row_ptr.device)
        res = new_result(csr.row_ptr.device)
        if ws is None:
            ws = workspace(csr.n, csr.m, flags, device=csr.row_ptr.device)
        _check(map_propagate(csr.n, csr.row_ptr, csr.col, csr.rrow_ptr, csr.rcol, acc, out, res, flags, ws,
                             stream), "map_propagate")
        return out, Result.from_tensor(res)


@dataclass
class DetectOut:
    result: Result
    trace: np.ndarray | None
    accepting_out: np.ndarray | None


def detect(csr: Csr, accepting0, trace_cap: int = 0, want_acc: bool = False, max_iterations: int = 0,
           flags: int = 0, ws=None, stream=None) -> DetectOut:
    """The MAP outer loop on the device; synchronizes to read the result."""
    dev = csr.row_ptr.device
    with _on(stream):
        acc = torch.as_tensor(accepting0, dtype=torch.uint8).to(dev).contiguous()
        res = new_result(dev)
        trace = torch.zeros((trace_cap, 3), dtype=torch.int64, device=dev) if trace_cap > 0 else None
        acc_out = torch.zeros(csr.n, dtype=torch.uint8, device=dev) if want_acc else None
        if ws is None:
            ws = workspace(csr.n, csr.m, flags, device=dev)
        _check(map_detect(csr.n, csr.row_ptr, csr.col, csr.rrow_ptr, csr.rcol, acc, res, trace, acc_out,
                          max_iterations, flags, ws, stream), "map_detect")
        r = Result.from_tensor(res)
        tr = None
        if trace is not None:
            tr = trace.cpu().numpy().view(np.uint64)[:min(r.iterations, trace_cap)].copy()
        return DetectOut(r, tr, acc_out.cpu().numpy() if acc_out is not None else None)


@dataclass
class LassoOut:
    status: int              # MAP_OK, MAP_ENOPATH, MAP_ENOSPC, MAP_ERANGE_DEV, MAP_EDEVICE
    stem_len: int            # edges init -> witness (0 without init), -1 if none
    cycle_len: int           # edges of the cycle through the witness, -1 if none
    path: np.ndarray | None  # ids: init, ..., witness, ..., witness (MAP_OK only)
    edges_scanned: int
    levels: int


def lasso(csr: Csr, witness: int, init: int = 0, cap: int | None = None, ws=None, stream=None) -> LassoOut:
    """Counterexample for ``witness``: shortest path from ``init`` (0: none), shortest cycle through it."""
    dev = csr.row_ptr.device
    cap = 2 * csr.n + 1 if cap is None else cap
    with _on(stream):
        path = torch.zeros(max(cap, 1), dtype=torch.int32, device=dev)
        res = torch.zeros(8, dtype=torch.int32, device=dev)
        if ws is None:
            ws = workspace(csr.n, csr.m, device=dev)
        _check(map_lasso(csr.n, csr.row_ptr, csr.col, witness, init, path[:cap], res, ws, stream), "map_lasso")
        a = res.cpu().numpy()
        status, s, c, plen = (int(x) for x in a[:4])
        scanned = int(a[4:6].view(np.int64)[0])
        return LassoOut(status, s, c, path[:plen].cpu().numpy() if status == MAP_OK else None, scanned,
                        int(a[6]))


@dataclass
class TrimOut:
    status: int
    kept: int
    accepting_kept: int
    rounds: int
    keep: torch.Tensor                 # device uint8[n]
    accepting: torch.Tensor | None     # device uint8[n]: accepting & keep


def trim(csr: Csr, accepting=None, ws=None, stream=None, sync: bool = True) -> TrimOut:
    """Relevance pruning on the device (needs the transposed CSR); synchronizes to read the counts."""
    if csr.rrow_ptr is None:
        raise ValueError("trim needs the transposed CSR (build_csr(..., transposed=True))")
    dev = csr.row_ptr.device
    with _on(stream):
        acc = None if accepting is None else torch.as_tensor(accepting, dtype=torch.uint8).to(dev).contiguous()
        keep = torch.empty(csr.n, dtype=torch.uint8, device=dev)
        acc_out = torch.empty(csr.n, dtype=torch.uint8, device=dev) if acc is not None else None
        res = torch.zeros(4, dtype=torch.int32, device=dev)
        if ws is None:
            ws = workspace(csr.n, csr.m, device=dev)
        _check(map_trim(csr.n, csr.row_ptr, csr.col, csr.rrow_ptr, csr.rcol, acc, keep, acc_out, res, ws,
                        stream), "map_trim")
        if not sync:
            return TrimOut(0, -1, -1, -1, keep, acc_out)
        a = res.cpu().numpy()
        return TrimOut(int(a[0]), int(a[1]), int(a[2]), int(a[3]), keep, acc_out)


# ------------------------------------------------------------------ batches

MAP_GRAPH_HUB_MASK = 0xFFFF
MAP_GRAPH_SYNC_SWEEPS = 0x10000
MAP_GRAPH_STREAM = 0x20000
MAP_GRAPH_FILTER = 0x40000
MAP_GRAPH_DIRECTION = 0x80000
GRAPH_DESC = np.dtype([("n", "<i4"), ("options", "<i4"), ("m", "<i8"), ("row_ptr", "<u8"), ("col", "<u8"),
                       ("accepting0", "<u8"), ("rrow_ptr", "<u8"), ("rcol", "<u8")])
assert GRAPH_DESC.itemsize == 56


class Batch:
    """Device descriptors, results and workspace for map_detect_batch.

    ``csrs`` and ``accs`` stay referenced so the device buffers outlive the
    launch.  Graphs are processed in the order given.  ``options`` (one int per
    graph, map_graph_desc.options) sets a graph's long-row threshold, fixpoint
    control, filtered sweeps and direction switch (the last needs the graph's
    transposed CSR); None leaves every graph at the defaults.
    """

    def __init__(self, csrs, accs, gang=None, flags: int = 0, device="cuda", options=None):
        self.csrs = list(csrs)
        self.accs = [torch.as_tensor(a, dtype=torch.uint8).to(device).contiguous() for a in accs]
        self.count = len(self.csrs)
        opts = np.zeros(self.count, np.int64) if options is None else np.asarray(options, np.int64)
        desc = np.zeros(self.count, GRAPH_DESC)
        for i, (c, a) in enumerate(zip(self.csrs, self.accs)):
            desc[i] = (c.n, int(opts[i]), c.m, c.row_ptr.data_ptr(), c.col.data_ptr(), a.data_ptr(),
                       c.rrow_ptr.data_ptr() if c.rrow_ptr is not None else 0,
                       c.rcol.data_ptr() if c.rcol is not None else 0)
        self.desc = torch.from_numpy(desc.view(np.uint8).copy()).to(device)
        self.gang = None if gang is None else torch.as_tensor(np.asarray(gang, np.int32)).to(device)
        self.total_n = int(sum(c.n for c in self.csrs))
        self.results = torch.zeros((self.count, 8), dtype=torch.int32, device=device)
        nbytes = map_batch_workspace_bytes(self.count, self.total_n, flags)
        if nbytes == 0:
            raise MapError(MAP_ERANGE, "map_batch_workspace_bytes")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.flags = flags
        self.stream = None   # stream of the last launch (None: torch's current stream)

    def launch(self, stream=None):
        _check(map_detect_batch(self.count, self.desc, self.gang, self.results, self.total_n, self.flags, self.ws,
                                stream), "map_detect_batch")
        self.stream = stream

    def read(self):
        """Results of the last launch (read on its stream, so they are final)."""
        with _on(self.stream):
            host = self.results.cpu()
        return [Result.from_tensor(host[i]) for i in range(self.count)]


# ------------------------------------------------------------ serving engine

class MapJob(ctypes.Structure):
    """struct map_job (include/mapcheck.h)."""
    _fields_ = [("n", ctypes.c_int32), ("gang", ctypes.c_int32), ("m", ctypes.c_int64),
                ("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("accepting0", ctypes.c_void_p), ("scratch", ctypes.c_void_p),
                ("tag", ctypes.c_uint64)]


class MapResultC(ctypes.Structure):
    """struct map_result (include/mapcheck.h)."""
    _fields_ = [("found", ctypes.c_int32), ("witness", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("status", ctypes.c_int32), ("sweeps", ctypes.c_int64), ("accepting_left", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


def map_job_scratch_bytes(n: int, m: int) -> int:
    return int(_lib.map_job_scratch_bytes(n, m))


class Engine:
    """A running map_engine: jobs are submitted and polled while it stays on the device.

    The engine kernel runs on its own stream until ``close()`` (or the idle
    bound).  ``submit`` takes tensors whose contents are final: the edge list
    and flags on the device or in pinned host memory, the CSR and scratch on
    the device; it keeps them referenced until the job is polled as done.
    """

    def __init__(self, max_jobs: int = 1024, workgroups: int = 0, idle_seconds: float = 60.0, flags: int = 0,
                 stream=None, device=None):
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        h = ctypes.c_void_p()
        _check(_lib.map_engine_create(max_jobs, workgroups, float(idle_seconds), flags,
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "map_engine_create")
        self._h = h
        self.workgroups = int(_lib.map_engine_workgroups(h))
        self._keep = {}

    def submit(self, n, src, dst, row_ptr, col, accepting0, scratch, gang: int = 1, tag: int = 0):
        """Post one job; returns its slot, or None when the engine is full (MAP_EBUSY)."""
        if self._h is None:
            raise MapError(MAP_EINVAL, "map_engine_submit")
        m = 0 if src is None else int(src.numel())
        job = MapJob(int(n), int(gang), m, _addr(src), _addr(dst), _addr(row_ptr), _addr(col), _addr(accepting0),
                     _addr(scratch), int(tag))
        slot = ctypes.c_int32(-1)
        rc = _lib.map_engine_submit(self._h, ctypes.byref(job), ctypes.byref(slot))
        if rc == MAP_EBUSY:
            return None
        _check(rc, "map_engine_submit")
        self._keep[slot.value] = (src, dst, row_ptr, col, accepting0, scratch)
        return slot.value

    def poll(self, slot: int):
        """Result of a finished job (its slot is freed), or None while it runs."""
        r = MapResultC()
        rc = _lib.map_engine_poll(self._h, int(slot), ctypes.byref(r))
        if rc == MAP_PENDING:
            return None
        self._keep.pop(slot, None)
        _check(rc, "map_engine_poll")
        return Result(r.found, r.witness, r.iterations, r.status, r.sweeps, r.accepting_left)

    def stop(self):
        if self._h is not None:
            _check(_lib.map_engine_stop(self._h), "map_engine_stop")

    def close(self):
        """Stop, wait for the engine kernel to exit, free it (idempotent)."""
        if self._h is not None:
            rc = _lib.map_engine_destroy(self._h)
            self._h = None
            self._keep.clear()
            _check(rc, "map_engine_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
