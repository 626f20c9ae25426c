"""Forward progress of the sort's look-back, shown on the CPU.

The single-sweep radix passes wait on other workgroups: a tile adds the
counts that the tiles before it publish.  `sort_lookback_emul.cpp` runs the
same protocol with threads as the resident workgroups (fewer than tiles,
random delays, look-back windows of 1 to 4 descriptors, eight passes on one
descriptor array).  With tile indices taken in start order, as the kernel
takes them, every exclusive prefix is exact and no wait reaches its bound.
With a fixed tile assignment instead, waits can form a cycle through a busy
worker; there the bound is what ends them, and the run still terminates.
"""
import os
import re
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def emul(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("lookback") / "sort_lookback_emul")
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-o", exe,
                    os.path.join(HERE, "sort_lookback_emul.cpp")], check=True)
    return exe


def _run(exe, mode):
    out = subprocess.run([exe, mode], check=True, capture_output=True, text=True,
                         timeout=240).stdout
    m = re.search(r"tiles_checked=(\d+) mismatches=(\d+) bound_hits=(\d+)", out)
    assert m, out
    return tuple(int(v) for v in m.groups())


def test_lookback_in_start_order_is_exact(emul):
    checked, mismatches, hits = _run(emul, "ordered")
    assert checked > 100000
    assert mismatches == 0
    assert hits == 0


def test_lookback_bound_ends_a_stalled_wait(emul):
    _, _, hits = _run(emul, "static")
    assert hits > 0
