"""Build libgf.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

    python -m paper_2306_11686_amd.build

Flags: -ffp-contract=off keeps every FP64 expression rounded exactly as
written (no FMA contraction), which the bit-exact parity of the stencil and
SpMV regions relies on; packed FP32 instructions are disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["gf_api.hip", "gf_kernels.hip", "gf_mlp.hip", "gf_heap.hip", "gf_noalloc.hip"]
LIB = os.path.join(HERE, "libgf.so")
ARCH = "gfx950"


# The sources the region kernels (persistent and per-region) are compiled
# from: the device code, its headers and the public header it includes.
KERNEL_SOURCES = ("csrc/gf_kernels.hip", "csrc/gf_device.h", "csrc/gf_internal.h", "csrc/gf_heap_dev.h",
                  "../include/gf.h")


def _code_only(text: str) -> str:
    """C/C++ source without comments and with whitespace collapsed, so that
    edits to comments do not count as changes to the code."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash() -> str:
    """Short hash of the code (comments aside) of the region kernels:
    measurements tied to those kernels (HBM traffic counters) record it and
    lapse when it changes."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.normpath(os.path.join(HERE, rel)), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-ffp-contract=off", "-mcode-object-version=5",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-result", "-Wno-unused-value", "-Wno-format-security",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    ]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + flags() + ["-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
