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
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libmdg.so")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
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


SOURCES = ("setup.cpp", "stage_launch.hip", "adjoint_kernel.hip", "api.hip")
# stage_kernel.hip is built once per (precision, order) instance
INSTANCES = [(r, p) for r in ("float", "double") for p in (1, 2, 3, 4)]


def build(verbose: bool = True) -> str:
    """Compiles every source (and every stage-kernel instance) to an object in
    parallel (each translation unit launches only its own kernels), then
    links the shared library."""
    generate()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = [os.path.join(BUILD, os.path.splitext(f)[0] + ".o") for f in SOURCES]
    cmds = [[HIPCC, *HIP_FLAGS, *inc, "-c", os.path.join(CSRC, f), "-o", o] for f, o in zip(SOURCES, objs)]
    for r, p in INSTANCES:
        o = os.path.join(BUILD, f"stage_kernel_{r}{p}.o")
        objs.append(o)
        cmds.append([HIPCC, *HIP_FLAGS, *inc, f"-DMDG_R={r}", f"-DMDG_P={p}", "-c",
                     os.path.join(CSRC, "stage_kernel.hip"), "-o", o])
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for fut in [ex.submit(_run, c) for c in cmds]:
            fut.result()
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
