import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_sessionstart(session):
    # Build the small C helpers (oracle, generators) if they are missing.
    import oracle
    import synth
    oracle.build(force=False)
    synth.build(force=False)


C_EXAMPLE = os.path.join(ROOT, "paper_0912_2555_amd", "examples", "detect")
C_EXAMPLE_TEST = "test_c_example_runs"
# Outcome of the C usage example (a child process), run once when the GPU test
# that checks it is selected, at the end of collection: before any test of
# this process touches the GPU, whatever order the test files run in.  (A
# second process's cooperative launch was refused once this process had made
# cooperative launches of its own.)
c_example_outcome = {}


def pytest_collection_finish(session):
    if not any(item.name == C_EXAMPLE_TEST for item in session.items):
        return
    import subprocess
    if not os.path.exists(C_EXAMPLE):
        c_example_outcome["error"] = "the C example is not built (python paper_0912_2555_amd/build.py)"
        return
    try:
        r = subprocess.run([C_EXAMPLE], capture_output=True, text=True, timeout=120)
        c_example_outcome.update(returncode=r.returncode, stdout=r.stdout, stderr=r.stderr)
    except subprocess.TimeoutExpired:
        c_example_outcome["error"] = "the C example did not finish within 120 s"


def read_golden(name):
    """Parse a tests/golden text fixture into {key: [rows of ints]}."""
    out = {}
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, *vals = line.split()
            out.setdefault(key, []).append([int(v) for v in vals])
    return out
