"""Code-generation guard for the asynchronous fixpoint control (CPU only).

The device code is compiled to gfx950 assembly here (hipcc cross-compiles) and
inspected:

- the bodies that run the asynchronous fixpoint control (the single-graph loop
  kernel and the gang body of the batch and the engine) must contain the grid
  barrier inline, never as a call.  Every build whose asynchronous body called
  the grid barrier out of line failed on the device (wrong verdicts on config
  2B with 16 gathers per lane; hangs of the early-detection kernel), and every
  build that inlined it passed; the mechanism is not known, so builds are held
  to the passing form.
- no asynchronous early-detection body is built (MAP_FLAG_EARLY runs with a
  barrier after every sweep).
"""
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_0912_2555_amd", "csrc", "mapcheck.hip")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Name prefixes of the asynchronous bodies: map_loop_kernel<true, false, ...>
# and the gang body of the batch and the engine.
ASYNC_BODIES = [
    "_ZN12_GLOBAL__N_115map_loop_kernelILb1ELb0E",
    "_ZN12_GLOBAL__N_119map_body_gang_asyncERKNS_8LoopArgsEPNS_5CtrlTILi256EEEii",
]


@pytest.fixture(scope="module")
def asm():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    import sys
    sys.path.insert(0, os.path.join(ROOT, "paper_0912_2555_amd"))
    try:
        import build as hipbuild  # the library's own compile flags
    finally:
        sys.path.pop(0)
    flags = [f for f in hipbuild.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "mapcheck.s")
        subprocess.check_call([HIPCC, *flags, "-I", os.path.join(ROOT, "include"), "--cuda-device-only",
                               "-S", "-o", out, SRC], stderr=subprocess.DEVNULL)
        return open(out).read()


def function_body(asm, prefix):
    """The assembly of the one function whose symbol starts with `prefix`."""
    found = re.findall(r"^(" + re.escape(prefix) + r"[\w.$]*):", asm, re.M)
    assert len(found) == 1, f"{prefix}: expected one function, found {found}"
    m = re.search(r"^" + re.escape(found[0]) + r":.*?^\.Lfunc_end", asm, re.S | re.M)
    return m.group(0)


def callees(body):
    """Names of the functions a body calls (each call loads its address pc-relative)."""
    return re.findall(r"s_add_u32\s+s\d+,\s*s\d+,\s*([\w.$]+)@rel32@lo", body)


@pytest.mark.parametrize("name", ASYNC_BODIES)
def test_async_bodies_inline_the_grid_barrier(asm, name):
    calls = callees(function_body(asm, name))
    assert calls, "expected at least the out-of-line sort call (parsing check)"
    assert not [c for c in calls if "grid_sync" in c], calls


def test_no_async_early_body_is_built(asm):
    assert "map_loop_kernelILb1ELb1E" not in asm
    assert "map_body_gang_async_early" not in asm


def test_callee_parser_sees_calls():
    body = ("f:\n\ts_getpc_b64 s[0:1]\n\ts_add_u32 s0, s0, _ZN12_GLOBAL__N_19grid_syncI@rel32@lo+4\n"
            "\ts_addc_u32 s1, s1, _ZN12_GLOBAL__N_19grid_syncI@rel32@hi+12\n\ts_swappc_b64 s[30:31], s[0:1]\n")
    assert callees(body) == ["_ZN12_GLOBAL__N_19grid_syncI"]
