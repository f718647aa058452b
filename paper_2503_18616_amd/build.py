"""Build libxpbd.so in-tree for gfx950 with hipcc.

    python -m paper_2503_18616_amd.build
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libxpbd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_SOURCES = ["xpbd_kernels.hip", "xpbd_runtime.hip", "mlp_kernels.hip", "warmstart_kernels.hip",
               "learned_runtime.hip", "tune_runtime.hip", "rl_kernels.hip", "rl_runtime.hip",
               "graph_runtime.hip", "lds_probe.hip", "norm_kernels.hip", "noalloc_runtime.hip"]
CXX_SOURCES = ["mesh_setup.cpp"]

# Packed FP32 instructions are kept out of every kernel.  The promotion budget
# lets both 32-register multiplier banks of the register-variant kernel live
# in VGPRs (otherwise one of them may be demoted to scratch memory).
HIP_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-mllvm", "-amdgpu-promote-alloca-to-vector-vgpr-ratio=2"]
# A multiplier bank in scratch would show up as at least 128 bytes per lane.
MAX_REG_KERNEL_SCRATCH = 96
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def _check_register_kernels(remarks: str):
    """Fail if a register-variant kernel keeps a multiplier bank in scratch."""
    name, scratch = None, {}
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name:
            scratch[name] = int(m.group(1))
    reg = {n: v for n, v in scratch.items()
           if "xpbd_step_reg_kernel" in n or "xpbd_substep_reg_kernel" in n}
    if not reg:
        raise RuntimeError("no resource-usage remarks for the register-variant kernels")
    bad = {n: v for n, v in reg.items() if v > MAX_REG_KERNEL_SCRATCH}
    if bad:
        raise RuntimeError(f"register-variant kernels use scratch {bad} bytes/lane: a "
                           "multiplier bank was not kept in VGPRs")


def _compile(name, verbose):
    """Compile one source into _build/; returns the object's path."""
    if name in CXX_SOURCES:
        obj = os.path.join(BUILD, name + ".o")
        _run(["g++", *CXX_FLAGS, "-c", os.path.join(SRC, name), "-o", obj], verbose)
        return obj
    obj = os.path.join(BUILD, name + ".o")
    cmd = [HIPCC, *HIP_FLAGS, "-c", os.path.join(SRC, name), "-o", obj]
    if name == "xpbd_kernels.hip":
        cmd.append("-Rpass-analysis=kernel-resource-usage")
        if verbose:
            print(" ".join(cmd), flush=True)
        out = subprocess.run(cmd, capture_output=True, text=True)
        if out.returncode != 0:
            sys.stderr.write(out.stderr)
            raise subprocess.CalledProcessError(out.returncode, cmd)
        _check_register_kernels(out.stderr)
    else:
        _run(cmd, verbose)
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source (several at once) and link the shared library;
    returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    names = HIP_SOURCES + CXX_SOURCES
    jobs = max(1, min(len(names), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        objects = list(pool.map(lambda n: _compile(n, verbose), names))
    tmp = LIB + f".tmp{os.getpid()}"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objects], verbose)
    os.replace(tmp, LIB)
    return LIB

if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
