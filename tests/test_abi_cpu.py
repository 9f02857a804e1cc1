"""The C-ABI library without a GPU: it loads, exports every declared symbol and
rejects bad arguments on the host before touching the device (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.environ.get("MAPCHECK_LIB") or os.path.join(ROOT, "paper_0912_2555_amd", "libmapcheck.so")
HEADER = os.path.join(ROOT, "include", "mapcheck.h")

MAP_OK, MAP_EINVAL, MAP_ERANGE, MAP_ENOSPC = 0, -1, -2, -3


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libmapcheck.so is not built (python paper_0912_2555_amd/build.py)")
    lib = ctypes.CDLL(LIB)
    vp, i32, i64, u32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t
    lib.map_workspace_bytes.argtypes = [i32, i64, u32]
    lib.map_workspace_bytes.restype = sz
    lib.map_build_csr.argtypes = [i32, i64, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.map_propagate.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, u32, vp, sz, vp]
    lib.map_detect.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, i32, vp, i32, u32, vp, sz, vp]
    lib.map_detect_noalloc.argtypes = [i32, vp, vp, vp, vp, vp, i32, vp, i32, u32, vp]
    lib.map_strerror.argtypes = [ctypes.c_int]
    lib.map_strerror.restype = ctypes.c_char_p
    return lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(map_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert names == ["map_batch_workspace_bytes", "map_build_csr", "map_detect", "map_detect_batch",
                     "map_detect_noalloc",
                     "map_engine_create", "map_engine_destroy", "map_engine_poll", "map_engine_stop",
                     "map_engine_submit", "map_engine_workgroups", "map_job_scratch_bytes", "map_lasso",
                     "map_phase_counters", "map_propagate", "map_strerror", "map_trim", "map_workspace_bytes"]
    for name in names:
        assert hasattr(lib, name), name


def test_header_compiles_as_c():
    import subprocess
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.c")
        with open(src, "w") as f:
            # Sizes and the descriptor's layout as the Python binding packs them.
            f.write('#include <stddef.h>\n#include "mapcheck.h"\nint main(void){ map_result r; map_job j; '
                    'map_lasso_result l; map_trim_result t; (void)r; (void)j; (void)l; (void)t; '
                    'return (int)sizeof(map_result) - 32 + (int)sizeof(map_job) - 72 '
                    '+ (int)sizeof(map_lasso_result) - 32 + (int)sizeof(map_trim_result) - 16 '
                    '+ (int)sizeof(map_graph_desc) - 56 + (int)offsetof(map_graph_desc, rrow_ptr) - 40 '
                    '+ (int)offsetof(map_graph_desc, rcol) - 48; }\n')
        subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                               "-o", os.path.join(d, "t"), src])
        assert subprocess.call([os.path.join(d, "t")]) == 0


def test_workspace_bytes(lib):
    a = lib.map_workspace_bytes(1000, 4000, 0)
    b = lib.map_workspace_bytes(1 << 20, 1 << 22, 0)
    assert a > 0 and b > a and b % 256 == 0
    assert b >= 5 * (1 << 20)  # packed values + working flags
    assert lib.map_workspace_bytes(0, 10, 0) == 0
    assert lib.map_workspace_bytes(-5, 10, 0) == 0
    assert lib.map_workspace_bytes(10, -1, 0) == 0
    assert lib.map_workspace_bytes(10, 1 << 31, 0) == 0


def test_host_side_errors_without_device(lib):
    fake = ctypes.c_void_p(0x1000)
    # sizes out of range
    assert lib.map_build_csr(0, 1, fake, fake, fake, fake, None, None, fake, fake, 1 << 20, None) == MAP_ERANGE
    assert lib.map_build_csr(5, -1, fake, fake, fake, fake, None, None, fake, fake, 1 << 20, None) == MAP_ERANGE
    # null pointers
    assert lib.map_build_csr(5, 3, None, fake, fake, fake, None, None, fake, fake, 1 << 20, None) == MAP_EINVAL
    assert lib.map_build_csr(5, 3, fake, fake, fake, fake, fake, None, fake, fake, 1 << 20, None) == MAP_EINVAL
    # workspace too small / misaligned
    assert lib.map_build_csr(5, 3, fake, fake, fake, fake, None, None, fake, fake, 16, None) == MAP_ENOSPC
    big = lib.map_workspace_bytes(5, 3, 0)
    assert lib.map_build_csr(5, 3, fake, fake, fake, fake, None, None, fake, ctypes.c_void_p(0x1004), big,
                             None) == MAP_ENOSPC
    assert lib.map_propagate(5, None, fake, None, None, fake, fake, fake, 0, fake, big, None) == MAP_EINVAL
    assert lib.map_propagate(5, fake, fake, None, None, fake, None, fake, 0, fake, big, None) == MAP_EINVAL
    assert lib.map_propagate(5, fake, fake, None, None, fake, fake, fake, 0x100, fake, big, None) == MAP_EINVAL
    # MAP_FLAG_DIRECTION needs the transposed CSR and excludes MAP_FLAG_PUSH
    assert lib.map_propagate(5, fake, fake, None, None, fake, fake, fake, 0x80, fake, big, None) == MAP_EINVAL
    assert lib.map_propagate(5, fake, fake, fake, fake, fake, fake, fake, 0x90, fake, big, None) == MAP_EINVAL
    assert lib.map_detect(0, fake, fake, None, None, fake, fake, None, 0, None, 0, 0, fake, big, None) == MAP_ERANGE
    assert lib.map_detect(5, fake, fake, None, None, None, fake, None, 0, None, 0, 0, fake, big, None) == MAP_EINVAL
    assert lib.map_detect(5, fake, fake, None, None, fake, None, None, 0, None, 0, 0, fake, big, None) == MAP_EINVAL
    assert lib.map_detect(5, fake, fake, None, None, fake, fake, fake, -1, None, 0, 0, fake, big, None) == MAP_EINVAL
    assert lib.map_detect(5, fake, fake, None, None, fake, fake, None, 0, None, 0, 0, fake, 8, None) == MAP_ENOSPC
    # MAP_FLAG_EARLY with MAP_FLAG_PUSH (frontier rounds) is refused before anything is enqueued
    assert lib.map_detect(5, fake, fake, fake, fake, fake, fake, None, 0, None, 0, 0x30, fake, big, None) == MAP_EINVAL
    assert lib.map_detect(5, fake, fake, fake, fake, fake, fake, None, 0, None, 0, 0x100, fake, big, None) == MAP_EINVAL
    assert lib.map_detect(5, fake, fake, None, None, fake, fake, None, 0, None, 0, 0x80, fake, big, None) == MAP_EINVAL
    assert lib.map_detect(5, fake, fake, fake, fake, fake, fake, None, 0, None, 0, 0x90, fake, big, None) == MAP_EINVAL


def test_noalloc_host_side_errors_without_device(lib):
    fake = ctypes.c_void_p(0x1000)
    max_n = 1 << 22  # MAP_NOALLOC_MAX_N
    # sizes beyond the fixed scratch, and empty graphs
    assert lib.map_detect_noalloc(max_n + 1, fake, fake, fake, fake, None, 0, None, 0, 0, None) == MAP_ERANGE
    assert lib.map_detect_noalloc(0, fake, fake, fake, fake, None, 0, None, 0, 0, None) == MAP_ERANGE
    # null pointers, unknown flags, frontier sweeps (no transposed CSR), negative trace capacity
    assert lib.map_detect_noalloc(5, None, fake, fake, fake, None, 0, None, 0, 0, None) == MAP_EINVAL
    assert lib.map_detect_noalloc(5, fake, fake, None, fake, None, 0, None, 0, 0, None) == MAP_EINVAL
    assert lib.map_detect_noalloc(5, fake, fake, fake, None, None, 0, None, 0, 0, None) == MAP_EINVAL
    assert lib.map_detect_noalloc(5, fake, fake, fake, fake, None, 0, None, 0, 0x100, None) == MAP_EINVAL
    assert lib.map_detect_noalloc(5, fake, fake, fake, fake, None, 0, None, 0, 0x80, None) == MAP_EINVAL
    assert lib.map_detect_noalloc(5, fake, fake, fake, fake, None, 0, None, 0, 0x10, None) == MAP_EINVAL
    assert lib.map_detect_noalloc(5, fake, fake, fake, fake, fake, -1, None, 0, 0, None) == MAP_EINVAL


def test_lasso_host_side_errors_without_device(lib):
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    lib.map_lasso.argtypes = [i32, vp, vp, i32, i32, vp, i32, vp, vp, sz, vp]
    fake = ctypes.c_void_p(0x1000)
    big = lib.map_workspace_bytes(5, 3, 0)
    assert lib.map_lasso(0, fake, fake, 1, 0, fake, 8, fake, fake, big, None) == MAP_ERANGE
    assert lib.map_lasso(5, None, fake, 1, 0, fake, 8, fake, fake, big, None) == MAP_EINVAL
    assert lib.map_lasso(5, fake, fake, 1, 0, fake, 8, None, fake, big, None) == MAP_EINVAL
    assert lib.map_lasso(5, fake, fake, 0, 0, fake, 8, fake, fake, big, None) == MAP_EINVAL   # witness 0
    assert lib.map_lasso(5, fake, fake, 6, 0, fake, 8, fake, fake, big, None) == MAP_EINVAL   # witness > n
    assert lib.map_lasso(5, fake, fake, 2, 6, fake, 8, fake, fake, big, None) == MAP_EINVAL   # init > n
    assert lib.map_lasso(5, fake, fake, 2, -1, fake, 8, fake, fake, big, None) == MAP_EINVAL
    assert lib.map_lasso(5, fake, fake, 2, 0, None, 8, fake, fake, big, None) == MAP_EINVAL   # path NULL, cap > 0
    assert lib.map_lasso(5, fake, fake, 2, 0, fake, -1, fake, fake, big, None) == MAP_EINVAL
    assert lib.map_lasso(5, fake, fake, 2, 0, fake, 8, fake, fake, 16, None) == MAP_ENOSPC
    assert lib.map_lasso(5, fake, fake, 2, 0, fake, 8, fake, ctypes.c_void_p(0x1004), big, None) == MAP_ENOSPC
    assert lib.map_strerror(-8).decode().startswith("no path")


def test_trim_host_side_errors_without_device(lib):
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    lib.map_trim.argtypes = [i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    f = ctypes.c_void_p(0x1000)
    big = lib.map_workspace_bytes(5, 3, 0)
    assert lib.map_trim(0, f, f, f, f, None, f, None, f, f, big, None) == MAP_ERANGE
    assert lib.map_trim(5, f, f, None, f, None, f, None, f, f, big, None) == MAP_EINVAL     # no transposed CSR
    assert lib.map_trim(5, f, f, f, f, None, None, None, f, f, big, None) == MAP_EINVAL     # keep_out NULL
    assert lib.map_trim(5, f, f, f, f, f, f, None, f, f, big, None) == MAP_EINVAL          # accepting w/o out
    assert lib.map_trim(5, f, f, f, f, None, f, f, f, f, big, None) == MAP_EINVAL          # out w/o accepting
    assert lib.map_trim(5, f, f, f, f, None, f, None, None, f, big, None) == MAP_EINVAL    # result NULL
    assert lib.map_trim(5, f, f, f, f, None, f, None, f, f, 64, None) == MAP_ENOSPC


def test_strerror(lib):
    for code in range(-6, 1):
        assert lib.map_strerror(code).decode()
    assert lib.map_strerror(99).decode() == "unknown status"


def test_batch_workspace_covers_filtered_scratch(lib):
    """The batch workspace grows with the graphs at least as fast as their
    scratch with MAP_GRAPH_FILTER does: values (4n) and flags (n), each
    256-aligned, and four 256-aligned bitmaps of ceil(n / 32) words."""
    lib.map_batch_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32]
    lib.map_batch_workspace_bytes.restype = ctypes.c_size_t
    al = lambda x: (x + 255) // 256 * 256
    per = lambda n: al(4 * n) + al(n) + 4 * al((n + 31) // 32 * 4)
    for ns in ([1000], [1, 2, 3], [10**6, 999_999, 31, 33], [257] * 100, [1 << 20] * 3):
        c = len(ns)
        grown = lib.map_batch_workspace_bytes(c, sum(ns), 0) - lib.map_batch_workspace_bytes(c, c, 0)
        assert grown >= sum(per(n) for n in ns) - c * per(1), ns
    # the least workspace (every graph n = 1) holds c scratches of n = 1
    assert lib.map_batch_workspace_bytes(7, 7, 0) >= 7 * per(1)


def test_engine_host_side_errors_without_device(lib):
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.map_job_scratch_bytes.argtypes = [i32, i64]
    lib.map_job_scratch_bytes.restype = ctypes.c_size_t
    lib.map_engine_create.argtypes = [i32, i32, ctypes.c_double, ctypes.c_uint32, vp, ctypes.POINTER(vp)]
    lib.map_engine_submit.argtypes = [vp, vp, ctypes.POINTER(i32)]
    lib.map_engine_poll.argtypes = [vp, i32, vp]
    lib.map_engine_stop.argtypes = [vp]
    lib.map_engine_destroy.argtypes = [vp]
    lib.map_engine_workgroups.argtypes = [vp]
    # values | flags | four bitmaps | scan partials | staged edges | transposed CSR, each 256-aligned
    assert lib.map_job_scratch_bytes(1000, 5000) == 4096 + 1024 + 4 * 256 + 1024 + 2 * 20224 + 4096 + 20224
    assert lib.map_job_scratch_bytes(0, 5) == 0
    assert lib.map_job_scratch_bytes(10, -1) == 0
    h = vp()
    assert lib.map_engine_create(16, 0, 1.0, 0, None, None) == MAP_EINVAL
    assert lib.map_engine_create(16, 0, 1.0, 0x100, None, ctypes.byref(h)) == MAP_EINVAL
    assert lib.map_engine_create(0, 0, 1.0, 0, None, ctypes.byref(h)) == MAP_ERANGE
    assert lib.map_engine_create(1 << 17, 0, 1.0, 0, None, ctypes.byref(h)) == MAP_ERANGE
    assert lib.map_engine_create(16, -1, 1.0, 0, None, ctypes.byref(h)) == MAP_ERANGE
    assert lib.map_engine_create(16, 0, 0.0, 0, None, ctypes.byref(h)) == MAP_ERANGE
    assert h.value is None
    slot = i32()
    assert lib.map_engine_submit(None, None, ctypes.byref(slot)) == MAP_EINVAL
    assert lib.map_engine_poll(None, 0, None) == MAP_EINVAL
    assert lib.map_engine_stop(None) == MAP_EINVAL
    assert lib.map_engine_destroy(None) == MAP_EINVAL
    assert lib.map_engine_workgroups(None) == 0
    assert lib.map_strerror(-7).decode().startswith("engine")
    assert lib.map_strerror(1).decode() == "job not finished yet"


def test_import_fails_without_the_library(tmp_path):
    """The binding has no fallback: a copy of the package without
    libmapcheck.so refuses to import."""
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_0912_2555_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_0912_2555_amd", "__init__.py"), pkg / "__init__.py")
    r = subprocess.run([sys.executable, "-c", "import paper_0912_2555_amd"], cwd=tmp_path, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "libmapcheck.so" in r.stderr


def test_product_code_does_not_use_the_oracle():
    """Only tests, the smoke check and the bench's CPU baseline may call the
    oracle: the package and its sources never name it."""
    pkg = os.path.join(ROOT, "paper_0912_2555_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".c", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\bimport\s+oracle\b|\bfrom\s+oracle\b|map_oracle", text), f
