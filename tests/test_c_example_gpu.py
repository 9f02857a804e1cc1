"""The C usage example (paper_0912_2555_amd/examples/detect.c): plain C against
the C ABI and the HIP runtime, no Python or torch in the process.  It checks
the results its two graphs fix (the worked example; a ring with a tail) and
exits with 0 when all match; the same values are checked here against the
oracle so that the example's own expectations are pinned too.

The example runs as a child process and launches cooperative kernels.  A
second process's cooperative launch was refused once this test process had
made cooperative launches of its own, so conftest.py runs the example at the
end of collection, before any test touches the GPU, and this test checks the
outcome it recorded; the order of the test files does not matter."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu



def test_expected_values_agree_with_the_oracle():
    g = synth.from_edges(5, [(1, 2), (2, 3), (3, 1), (3, 4), (4, 5)], [2, 4, 5])
    d = oracle.map_detect(g)
    lz = oracle.lasso(g, d.witness, 1)
    assert (d.found, d.witness, d.iterations, lz.stem_len, lz.cycle_len) == (1, 2, 3, 1, 3)
    n, ring = 1000, 600
    src = np.arange(1, n + 1, dtype=np.int32)
    dst = np.array([1 if v in (ring, n) else v + 1 for v in range(1, n + 1)], np.int32)
    acc = (np.arange(1, n + 1) % 7 == 0).astype(np.uint8)
    g = synth.Graph(n=n, src=src, dst=dst, acc=acc)
    d = oracle.map_detect(g)
    lz = oracle.lasso(g, d.witness, ring + 1)
    assert (d.found, d.witness, d.iterations, lz.stem_len, lz.cycle_len) == (1, 595, 1, 994, 600)


def test_c_example_runs():
    from conftest import c_example_outcome as out
    assert "error" not in out, out.get("error")
    assert out, "the C example was not run at the end of collection"
    print(out["stdout"], out["stderr"], flush=True)
    assert out["returncode"] == 0
    lines = out["stdout"].strip().splitlines()
    assert len(lines) == 2 and all(line.endswith(" ok") for line in lines)
