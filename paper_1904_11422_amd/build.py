"""Build libepic.so (the C ABI of include/epic.h) for gfx950 with hipcc.

    python -m paper_1904_11422_amd.build [--verbose]
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libepic.so")
SOURCES = [os.path.join(PKG, "csrc", "epic.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def hipcc_command(out: str = LIB, extra=()) -> list:
    return [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            # packed FP32 instructions stay off (see the design notes)
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # matrix-core results in ordinary VGPRs: the split-precision
            # epilogue reads them without accumulator-register moves
            "-mllvm", "-amdgpu-mfma-vgpr-form",
            "-I", os.path.join(ROOT, "include"), *extra, "-o", out, *SOURCES]


def build(verbose: bool = False, extra=()) -> str:
    cmd = hipcc_command(extra=extra)
    tmp = LIB + ".tmp"
    cmd[cmd.index(LIB)] = tmp
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libepic.so")
    if verbose and r.stderr.strip():
        sys.stderr.write(r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="--verbose" in sys.argv)
    print(LIB)
