"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only).

libmapcheck is rebuilt with the sanitizers on its host code only (each
-fsanitize is passed to the host compilation alone, with -Xarch_host; the
device code is built as usual and never runs here), and the host-side ABI
tests -- every export, the workspace, batch and job sizes, and the argument
checks that reject bad calls before any device work -- run against that build
in a child Python process (MAPCHECK_LIB selects it; the compiler's ASan runtime
is preloaded, leak checking off because the interpreter is not instrumented).
Any invalid access or undefined behaviour aborts the child, so the test fails.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


def _asan_runtime():
    found = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    asan = _asan_runtime()
    if not os.path.exists(HIPCC) or asan is None:
        pytest.skip("no HIP compiler or no ASan runtime")
    lib = str(tmp_path / "libmapcheck_san.so")
    cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-Xarch_host", "-fno-omit-frame-pointer", "-shared-libsan",
           "-I", os.path.join(ROOT, "include"), "-o", lib,
           os.path.join(ROOT, "paper_0912_2555_amd", "csrc", "mapcheck.hip")]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert b.returncode == 0, b.stderr[-3000:]
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_" in syms and "__ubsan_" in syms
    env = dict(os.environ)
    env["MAPCHECK_LIB"] = lib
    env["LD_PRELOAD"] = asan + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    # (the one ABI test that needs the package to find no library is left out)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        "-k", "not import_fails_without_the_library", "tests/test_abi_cpu.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert " passed" in r.stdout, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, tail
