import ctypes
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _keep_freed_memory():
    """The oracle allocates the arrays of every stage of every step afresh.  By default
    glibc serves blocks of a few MB with mmap and unmaps them on free, so each step
    faults in fresh zeroed pages; raising the mmap and trim thresholds keeps freed
    blocks in the heap for the next step (3-4x faster oracle runs on 256^2 meshes)."""
    try:
        libc = ctypes.CDLL("libc.so.6")
    except OSError:
        return
    M_TRIM_THRESHOLD, M_MMAP_THRESHOLD = -1, -3
    libc.mallopt(M_MMAP_THRESHOLD, 1 << 30)
    libc.mallopt(M_TRIM_THRESHOLD, (1 << 31) - 1)


_keep_freed_memory()


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long oracle pins, enabled with LBFV_SLOW_PINS=1")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("LBFV_SLOW_PINS") == "1":
        return
    skip = pytest.mark.skip(reason="long oracle pin; set LBFV_SLOW_PINS=1 to run")
    for it in items:
        if "slow" in it.keywords:
            it.add_marker(skip)
