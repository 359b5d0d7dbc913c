"""Build libumesh.so (host planner + gfx950 HIP kernels + C ABI) in-tree.

    python -m paper_1802_03749_amd.build

Host-only C++ (reordering, planning) is compiled with g++; files that use
the HIP runtime or hold kernels are compiled with hipcc for gfx950.  Objects
go to paper_1802_03749_amd/_build/, the library to
paper_1802_03749_amd/libumesh.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libumesh.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HOST_SOURCES = ["reorder.cpp", "planner.cpp", "planner_step.cpp"]
HIP_SOURCES = ["api.cpp", "kernels_lf2d.hip", "kernels_hex.hip", "kernels_step.hip",
               "kernels_util.hip"]

# Device code is built without packed-FP32 instructions (explicitly disabled
# feature) and without fast-math: division and sqrt stay IEEE-correct.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics", "-Wall", "-Wno-unused-result"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), file=sys.stderr, flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


def build(verbose: bool = False, jobs: int = 8) -> str:
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I", INCLUDE, "-I", CSRC]
    cmds = []
    objs = []
    for s in HOST_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        cmds.append(["g++", *HOST_FLAGS, *inc, "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in HIP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        lang = ["-x", "hip"]
        cmds.append([hipcc, *HIP_FLAGS, *inc, *lang, "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs,
          f"-L{ROCM}/lib", "-lamdhip64", "-Wl,--no-undefined"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
