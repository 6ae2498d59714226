"""The gfx950 code object inside liblbfv.so: extraction and per-kernel machine-code digests.

A counter profile describes one compiled kernel.  ``kernel_isa_sha256`` hashes that kernel's
machine code and its kernel descriptor (registers, LDS, scratch), so a measurement can be
tied to the exact binary it was taken on: a change elsewhere in the sources leaves the digest
alone, a change to the kernel's code does not.  Uses the ROCm LLVM tools; returns None when
they are missing.
"""
from __future__ import annotations

import hashlib
import os
import struct
import subprocess
import tempfile

LLVM = "/opt/rocm/llvm/bin"
TARGET = "hipv4-amdgcn-amd-amdhsa--gfx950"


def extract(lib: str) -> bytes | None:
    """The gfx950 ELF code object bundled in `lib`'s .hip_fatbin section."""
    objcopy, bundler = os.path.join(LLVM, "llvm-objcopy"), os.path.join(LLVM, "clang-offload-bundler")
    if not (os.path.exists(objcopy) and os.path.exists(bundler) and os.path.exists(lib)):
        return None
    with tempfile.TemporaryDirectory() as d:
        fat, host, co = (os.path.join(d, n) for n in ("fatbin", "host.so", "device.co"))
        try:
            subprocess.run([objcopy, f"--dump-section=.hip_fatbin={fat}", lib, host], check=True,
                           capture_output=True)
            subprocess.run([bundler, "--unbundle", "--type=o", f"--targets={TARGET}", f"--input={fat}",
                            f"--output={co}"], check=True, capture_output=True)
        except (OSError, subprocess.CalledProcessError):
            return None
        with open(co, "rb") as f:
            return f.read()


def symbols(elf: bytes) -> dict:
    """name -> (file offset, size) of every sized symbol of a little-endian ELF64 file."""
    shoff, = struct.unpack_from("<Q", elf, 0x28)
    shentsize, shnum = struct.unpack_from("<HH", elf, 0x3A)
    secs = [struct.unpack_from("<IIQQQQIIQQ", elf, shoff + i * shentsize) for i in range(shnum)]
    out = {}
    for sec in secs:
        if sec[1] != 2:                      # SHT_SYMTAB
            continue
        strtab = secs[sec[6]]
        for k in range(sec[5] // 24):
            name_off, _info, _other, shndx, value, size = struct.unpack_from("<IBBHQQ", elf, sec[4] + k * 24)
            if size == 0 or shndx == 0 or shndx >= len(secs):
                continue
            start = strtab[4] + name_off
            name = elf[start:elf.index(b"\0", start)].decode()
            host = secs[shndx]
            out[name] = (value - host[3] + host[4], size)
    return out


def kernel_isa_sha256(lib: str, kernel: str) -> str | None:
    """SHA-256 over the machine code of `kernel` (mangled name) and its kernel descriptor."""
    elf = extract(lib)
    if elf is None:
        return None
    return _digest(elf, symbols(elf), kernel)


def kernel_digests(lib: str) -> dict | None:
    """kernel_isa_sha256 of every kernel in `lib`, from one extraction: {mangled name: digest}."""
    elf = extract(lib)
    if elf is None:
        return None
    syms = symbols(elf)
    return {k: _digest(elf, syms, k) for k in syms if not k.endswith(".kd") and k + ".kd" in syms}


def _digest(elf: bytes, syms: dict, kernel: str) -> str | None:
    if kernel not in syms or kernel + ".kd" not in syms:
        return None
    h = hashlib.sha256()
    off, size = syms[kernel]
    h.update(elf[off:off + size])
    # the 64-byte kernel descriptor, less its position-dependent field (bytes 16..23: the
    # offset from the descriptor to the code entry, which moves when other kernels change)
    off, size = syms[kernel + ".kd"]
    kd = bytearray(elf[off:off + size])
    kd[16:24] = bytes(8)
    h.update(bytes(kd))
    return h.hexdigest()
