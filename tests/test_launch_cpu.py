"""Launch-shape guard over the library source (CPU only).

grid_for() caps a launch at 65,536 workgroups, so every kernel launched with
a grid from it must step over its range in grid strides (a loop that advances
by gridDim.x * blockDim.x); a kernel that assumed one thread per element would
leave everything past 2^24 elements of a 256-thread launch untouched.
"""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_0912_2555_amd", "csrc", "mapcheck.hip")


def kernel_body(src, name):
    m = re.search(r"__global__ void(?:\s+__launch_bounds__\([^)]*\))?\s+" + re.escape(name) + r"\s*\(", src)
    assert m, name
    i = src.index("{", m.end())
    depth = 0
    for j in range(i, len(src)):
        depth += {"{": 1, "}": -1}.get(src[j], 0)
        if depth == 0:
            return src[i:j + 1]
    raise AssertionError(name)


def test_capped_launches_stride_over_their_range():
    src = open(SRC).read()
    names = sorted(set(re.findall(r"hipLaunchKernelGGL\((\w+),\s*dim3\(grid_for\(", src)))
    assert "csr_order_rows" in names and "csr_scatter" in names
    for name in names:
        body = kernel_body(src, name)
        assert re.search(r"gridDim\.x\s*\*\s*blockDim\.x", body), f"{name} has no grid-stride loop"


def test_grid_cap_is_what_the_guard_assumes():
    src = open(SRC).read()
    m = re.search(r"inline unsigned grid_for\(int64_t work, int threads\) \{(.*?)\n\}", src, re.S)
    assert m and "65536" in m.group(1)
