"""The oracle's pins under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The plain C oracle is rebuilt with -fsanitize=address,undefined (host code,
gcc) and the pin tests of every oracle function run against that build in a
child Python process (ORACLE_LIB selects it; the ASan runtime is preloaded
ahead of anything already preloaded, leak checking off because the Python
interpreter itself is not instrumented).  Any invalid access or undefined
behaviour aborts the child, so the test fails.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_TESTS = ["tests/test_oracle_pins.py", "tests/test_lasso_oracle.py", "tests/test_trim_oracle.py"]


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    import oracle
    try:
        lib = oracle.build_sanitized(str(tmp_path))
        asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    except (OSError, subprocess.CalledProcessError) as e:
        pytest.skip(f"no sanitizer toolchain: {e}")
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("libasan not found")
    env = dict(os.environ)
    env["ORACLE_LIB"] = lib
    env["LD_PRELOAD"] = asan + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    # the child loads the instrumented build, and ASan's runtime is in the process
    probe = subprocess.run([sys.executable, "-c", "import oracle; oracle._load(); print(sorted(oracle._libs))"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert probe.returncode == 0 and lib in probe.stdout, probe.stdout + probe.stderr
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_" in syms and "__ubsan_" in syms
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        *PIN_TESTS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert " passed" in r.stdout, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, tail
