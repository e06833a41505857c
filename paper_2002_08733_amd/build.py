"""Build libmdg.so for gfx950 in-tree.

Steps: compile and run the reference-operator generator (host C++), then
compile the host setup, the kernels and the C ABI with hipcc into
``paper_2002_08733_amd/libmdg.so``.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libmdg.so")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 VALU ops are disabled for every HIP source of this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-parameter",
]


def _run(cmd, **kw):
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, **kw)


def generate():
    os.makedirs(BUILD, exist_ok=True)
    gen = os.path.join(BUILD, "gen_refops")
    _run(["g++", "-O2", "-std=c++17", "-o", gen, os.path.join(CSRC, "gen_refops.cpp")])
    _run([gen, os.path.join(CSRC, "refops_gen.h"), os.path.join(CSRC, "refops_dev_gen.h"),
          os.path.join(CSRC, "refops_gen.txt")])


def build(verbose: bool = True) -> str:
    generate()
    srcs = [os.path.join(CSRC, f) for f in ("setup.cpp", "stage_kernel.hip", "adjoint_kernel.hip", "api.hip")]
    tmp = LIB + ".tmp"
    _run([HIPCC, *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, *srcs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
