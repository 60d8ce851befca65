"""GPU test of the PRUNE_DEBUG build (libprune_hip_debug.so): its
bookkeeping kernels check every FIFO after each counter update (reachable
block state, token occupancy within Eq. 2's capacity, counters that only
grow) and a failed check makes prune_graph_sync return E_RULE.  The graph
tests (per-firing, batched and pipelined rounds, delays of every alignment,
routed, unfused and pixel graphs, host streaming) and the stop tests run in
one child process on that build: every check holds and every result still
matches the oracle."""
import os
import subprocess
import sys

import pytest

from gpu_util import announce

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEBUG_LIB = os.path.join(ROOT, "paper_1802_06625_amd", "libprune_hip_debug.so")


@pytest.mark.timeout(600)
def test_graph_tests_hold_every_invariant_check():
    announce("debug build: graph and stop tests")
    assert os.path.exists(DEBUG_LIB), "libprune_hip_debug.so is missing: run __graft_entry__.build()"
    env = dict(os.environ, PRUNE_DEBUG_LIBRARY="1")
    # the full-size graphs are left to the release build: the checks are the
    # same at any size, and the small graphs reach every bookkeeping path
    cmd = [sys.executable, "-u", "-m", "pytest", "-x", "-m", "gpu", "-p", "no:cacheprovider",
           "--timeout", "240", "--timeout-method", "thread", "-k", "not full_size and not 1080p",
           os.path.join(ROOT, "tests", "test_gpu_graph.py"), os.path.join(ROOT, "tests", "test_gpu_stop.py")]
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = "\n".join((res.stdout + res.stderr).splitlines()[-30:])
    assert res.returncode == 0, tail
    assert "debug build loaded" in res.stdout, tail
    assert " passed" in res.stdout and " failed" not in res.stdout, tail
