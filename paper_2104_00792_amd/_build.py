"""Compile the HashGraph HIP library (libhg.so) for gfx950, in-tree."""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libhg.so")
SOURCES = ["hg_kernels.hip", "hg_split.hip", "hg_api.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose: bool = False) -> str:
    """Build libhg.so next to this file and return its path."""
    tmp = LIB + ".tmp"
    cmd = [
        HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O3", "-std=c++17",
        "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
        # Code object v5: loadable by the HIP runtime that ships with torch.
        "-mcode-object-version=5",
        # Packed FP32 instructions stay off: this path has no floating point,
        # and the flag keeps the compiler from forming them anywhere.
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", INCLUDE, "-I", CSRC,
        *[os.path.join(CSRC, s) for s in SOURCES],
        "-o", tmp,
    ]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
