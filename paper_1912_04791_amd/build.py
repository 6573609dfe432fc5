"""Build libdsve.so (HIP kernels for gfx950 + the C ABI host code) in-tree with hipcc.

    python -m paper_1912_04791_amd.build          # or build() from Python

The library lands next to this file as ``libdsve.so``; the ctypes binding in
``dsve.py`` loads it from there and raises if it is missing.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdsve.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

ARCH = os.environ.get("DSVE_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are switched off for all device code.
DEVICE_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall"]

SOURCES = {
    "dsve_kernels.hip": DEVICE_FLAGS,
    "dsve_api.cpp": HOST_FLAGS,
}


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm toolchain required to build libdsve.so)")


def build(verbose: bool = False, extra_device_flags=None, out: str | None = None) -> str:
    """Compile every source and link libdsve.so (or `out`); always recompiles."""
    cc = hipcc()
    lib = out or LIB
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src, flags in SOURCES.items():
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        fl = list(flags)
        if src.endswith(".hip") and extra_device_flags:
            fl += list(extra_device_flags)
        cmd = [cc, *fl, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = f"{lib}.{os.getpid()}.tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
