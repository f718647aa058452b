"""Build libxpbd.so in-tree for gfx950 with hipcc.

    python -m paper_2503_18616_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libxpbd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_SOURCES = ["xpbd_kernels.hip", "xpbd_runtime.hip"]
CXX_SOURCES = ["mesh_setup.cpp"]

# Packed FP32 instructions are kept out of every kernel.
HIP_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    """Compile every source and link the shared library; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    objects = []
    for name in HIP_SOURCES:
        obj = os.path.join(BUILD, name + ".o")
        _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(SRC, name), "-o", obj], verbose)
        objects.append(obj)
    for name in CXX_SOURCES:
        obj = os.path.join(BUILD, name + ".o")
        _run(["g++", *CXX_FLAGS, "-c", os.path.join(SRC, name), "-o", obj], verbose)
        objects.append(obj)
    tmp = LIB + f".tmp{os.getpid()}"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objects], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
