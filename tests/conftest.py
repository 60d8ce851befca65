import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_report_header(config):
    # a run on the PRUNE_DEBUG build says so, after checking the build's flag
    if os.environ.get("PRUNE_DEBUG_LIBRARY", "0") not in ("", "0"):
        from paper_1802_06625_amd import _lib as L
        flags = L.lib().prune_build_flags()
        assert flags & L.BUILD_DEBUG, f"PRUNE_DEBUG_LIBRARY set but the loaded library has flags {flags}"
        return f"debug build loaded: {L.LIB_PATH}"
    return None
