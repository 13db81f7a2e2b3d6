"""Build the HIP library libedge_lts.so (gfx950) in-tree.

Steps: compile and run the reference-matrix generator (host C++), then compile
the HIP kernels and the host library with hipcc and link the shared object.
Object files are compiled in parallel; everything lands under
paper_2202_10313_amd/_build and paper_2202_10313_amd/lib.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIBDIR = os.path.join(HERE, "lib")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(LIBDIR, "libedge_lts.so")
ORDERS = ["2", "3", "4", "5"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", CSRC, "-I", INCLUDE]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + os.path.basename(cmd[0]))
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    os.makedirs(os.path.join(CSRC, "generated"), exist_ok=True)
    gen = os.path.join(BUILD, "gen_refmats")
    _run(["g++", "-O2", "-std=c++17", "-o", gen, os.path.join(CSRC, "gen_refmats.cpp"),
          os.path.join(CSRC, "basis.cpp")])
    _run([gen, os.path.join(CSRC, "generated", "refmats.h")] + ORDERS)
    units = [("kernels.hip", "kernels.o"), ("adjoint.hip", "adjoint.o"), ("host.cpp", "host.o"),
             ("basis.cpp", "basis.o"), ("noalloc.hip", "noalloc.o"),
             ("materials.hip", "materials.o"), ("debug.hip", "debug.o")]

    def compile_unit(u):
        src, obj = u
        extra = ["-x", "hip"] if src.endswith(".hip") else []
        _run([HIPCC] + HIPFLAGS + extra + ["-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, obj)])
        return obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_unit, units))
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [os.path.join(BUILD, o) for o in objs])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
