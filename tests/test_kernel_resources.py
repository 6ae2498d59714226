"""Register and scratch use of the built kernels, read from the gfx950 code object inside
liblbfv.so (no GPU needed).  A march whose state lands in scratch memory, or a helper that
the compiler stops inlining (it then keeps the march's state on the stack), runs several
times slower with identical results, so no parity test notices; this test does."""
import os
import re
import subprocess

import pytest

from paper_1511_00242_amd import lbfv as L

LLVM = "/opt/rocm/llvm/bin"
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"

# Kernels allowed to use scratch memory or to spill vector registers, with the reason.
ALLOWED = {
    # two time steps per launch in FP64 on a single wave per batch item: both time levels'
    # rows live in one wave; the pair form (batch2p_kernel) is the one that fits
    "_ZN4lbfv13batch2_kernelIddLi0ELb1EEEvPKNS_10StepParamsIT_EEPKNS_9BatchItemEii",
}


def kernel_metadata(tmp_path):
    tools = [os.path.join(LLVM, t) for t in ("llvm-objcopy", "clang-offload-bundler", "llvm-readelf")]
    if not all(os.path.exists(t) for t in tools):
        pytest.skip("ROCm LLVM tools not found")
    lib = L._LIB_PATH
    if not os.path.exists(lib):
        pytest.skip("liblbfv.so is not built")
    fat, dummy, co = tmp_path / "fatbin", tmp_path / "host.so", tmp_path / "gfx950.co"
    subprocess.run([tools[0], f"--dump-section=.hip_fatbin={fat}", lib, str(dummy)], check=True)
    subprocess.run([tools[1], "--unbundle", "--type=o", f"--targets={TARGET}", f"--input={fat}",
                    f"--output={co}"], check=True)
    notes = subprocess.run([tools[2], "--notes", str(co)], check=True, capture_output=True, text=True).stdout
    # the kernel records of the AMDGPU metadata note, one YAML mapping each
    out = {}
    for rec in re.split(r"\n  - ", notes)[1:]:
        name = re.search(r"\.name:\s+(\S+)", rec)
        if not name or not name.group(1).startswith("_ZN4lbfv"):
            continue
        def field(k):
            m = re.search(r"\." + k + r":\s+(\d+)", rec)
            return int(m.group(1)) if m else 0
        out[name.group(1)] = {k: field(k) for k in ("private_segment_fixed_size", "vgpr_spill_count",
                                                      "vgpr_count", "sgpr_count")}
    return out


def test_no_kernel_uses_scratch_memory(tmp_path):
    md = kernel_metadata(tmp_path)
    assert len(md) > 100, "expected every step, batch and auxiliary kernel in the code object"
    assert any("step2p_kernel" in k for k in md) and any("batch2p_kernel" in k for k in md)
    bad = {k: v for k, v in md.items()
           if k not in ALLOWED and (v["private_segment_fixed_size"] or v["vgpr_spill_count"])}
    assert not bad, bad


def test_pair_kernels_fit_two_waves_per_simd(tmp_path):
    # 512 vector registers per SIMD lane: the FP64 pair and chain kernels (the headline and
    # the forms with sides) must stay at or below 256 so that two waves share a SIMD
    md = kernel_metadata(tmp_path)
    for k, v in md.items():
        if "step2p_kernelIdd" in k or "step2bp_kernelIdd" in k or "stepc_kernelIdd" in k:
            assert v["vgpr_count"] <= 256, (k, v)


def test_kernel_digest_identifies_the_binary_kernel():
    # the digest bench.py ties a counter profile to: stable, and distinct per kernel
    from paper_1511_00242_amd import codeobj
    lib = L._LIB_PATH
    if not os.path.exists(lib):
        pytest.skip("liblbfv.so is not built")
    head = "_ZN4lbfv13step2p_kernelIddLi0ELb0EEEvNS_10StepParamsIT_EEiiii"
    bkg = "_ZN4lbfv13step2p_kernelIddLi1ELb0EEEvNS_10StepParamsIT_EEiiii"
    h1, h2, h3 = (codeobj.kernel_isa_sha256(lib, k) for k in (head, head, bkg))
    if h1 is None:
        pytest.skip("ROCm LLVM tools not found")
    assert re.fullmatch(r"[0-9a-f]{64}", h1) and h1 == h2 and h1 != h3
    assert codeobj.kernel_isa_sha256(lib, "no_such_kernel") is None
