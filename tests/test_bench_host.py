"""Host logic of the benchmark (no GPU): the committed counter profile that bench.py turns
into the roofline's measured traffic must describe the kernel and launch shape it times, and
any other shape or kernel must get no traffic figure."""
import os

import pytest

import bench
from paper_1511_00242_amd import codeobj
from paper_1511_00242_amd import lbfv as L


def _need_digest():
    if not os.path.exists(L._LIB_PATH):
        pytest.skip("liblbfv.so is not built")
    if codeobj.kernel_isa_sha256(L._LIB_PATH, bench.HEADLINE_KERNEL) is None:
        pytest.skip("ROCm LLVM tools not found")


def test_committed_traffic_profile_describes_the_timed_kernel():
    # a change to the headline kernel's machine code needs a new counter profile
    _need_digest()
    gbs, b = bench.profiled_traffic(bench.HEADLINE_TILE, bench.HEADLINE_TIME_BLOCK, 0.25, bench.HEADLINE_PAIRS)
    assert b is not None, "profiles/traffic_dugks_fp64_taylor_green_4096.txt is stale for the built kernel"
    # FETCH_SIZE and WRITE_SIZE scaled by the device-copy calibration: at least the state read
    # and written once per launch (2 x 9 x 8 B x 4096^2), at most the bytes of every step
    state = 2 * 9 * 8 * 4096 * 4096
    assert state < b < bench.HEADLINE_TIME_BLOCK * state
    assert gbs == pytest.approx(b / (bench.HEADLINE_TIME_BLOCK * 0.25e-3) / 1e9)


def test_traffic_withheld_for_another_launch_shape():
    _need_digest()
    rows, wpb = bench.HEADLINE_TILE
    tb = bench.HEADLINE_TIME_BLOCK
    assert bench.profiled_traffic((rows + 1, wpb), tb, 0.25, bench.HEADLINE_PAIRS) == (None, None)
    assert bench.profiled_traffic((rows, wpb), 1 if tb != 1 else 2, 0.25, bench.HEADLINE_PAIRS) == (None, None)
    assert bench.profiled_traffic((rows, wpb), tb, 0.25, 1 - bench.HEADLINE_PAIRS) == (None, None)


def test_traffic_withheld_for_another_kernel(monkeypatch):
    _need_digest()
    other = "_ZN4lbfv13step2p_kernelIddLi0ELb0EEEvNS_10StepParamsIT_EEiiii"
    monkeypatch.setattr(bench, "HEADLINE_KERNEL", other)
    assert bench.profiled_traffic(bench.HEADLINE_TILE, bench.HEADLINE_TIME_BLOCK, 0.25,
                                  bench.HEADLINE_PAIRS) == (None, None)


def test_every_counter_profile_describes_a_built_kernel():
    # each committed rocprofv3 summary names the machine-code digest of the kernel it measured;
    # all of them must still be kernels of the built library
    import re
    _need_digest()
    built = set(codeobj.kernel_digests(L._LIB_PATH).values())
    pdir = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles")
    seen = 0
    for name in sorted(os.listdir(pdir)):
        for h in set(re.findall(r"\b[0-9a-f]{64}\b", open(os.path.join(pdir, name)).read())):
            seen += 1
            assert h in built, f"{name}: profiled kernel {h[:12]} is not in the built library"
    assert seen >= 5
