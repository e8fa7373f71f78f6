"""Compile the HIP/C++ library libqforte_mi355x.so in-tree for gfx950.

    python paper_2108_04413_amd/build.py

(run it as a script: importing the package loads the library it builds).

Steps: hipcc compiles the device file (kernels + C-ABI entry points), g++
compiles the host builder, hipcc links the shared library next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libqforte_mi355x.so")
ARCH = os.environ.get("QF_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-result"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = True) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    dev_o = os.path.join(OUT_DIR, "qf_device.o")
    bat_o = os.path.join(OUT_DIR, "qf_batch.o")
    bld_o = os.path.join(OUT_DIR, "qf_builder.o")
    sec_o = os.path.join(OUT_DIR, "qf_sector.o")
    _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "qf_device.hip"), "-o", dev_o])
    _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "qf_batch.hip"), "-o", bat_o])
    _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "qf_sector.hip"), "-o", sec_o])
    _run(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, "qf_builder.cpp"), "-o", bld_o])
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, dev_o, bat_o, sec_o, bld_o])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
