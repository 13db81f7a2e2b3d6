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


# Host code under AddressSanitizer and UndefinedBehaviorSanitizer (a CPU
# test aid): the host C++ (host.cpp, basis.cpp) compiled with g++ and both
# sanitizers, any error fatal, linked with the HIP objects of the regular
# build (device code is not instrumented); and the reference-matrix
# generator built the same way.  The results are keyed by a hash of the
# sources, so an unchanged tree is not rebuilt.  Load the library with the
# ASan runtime preloaded (LD_PRELOAD=<sanitizer_runtime()>) and
# EDG_LIBRARY pointing at it.
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def sanitizer_runtime() -> str:
    return _run(["g++", "-print-file-name=libasan.so"]).stdout.strip()


def build_sanitized_host() -> dict:
    import hashlib
    hip_names = ("kernels.o", "adjoint.o", "debug.o", "materials.o", "noalloc.o")
    if not (os.path.exists(LIB) and all(os.path.exists(os.path.join(BUILD, o)) for o in hip_names)):
        build()
    san = os.path.join(BUILD, "san")
    os.makedirs(san, exist_ok=True)
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".cpp", ".hpp")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + f.read())
    with open(os.path.join(INCLUDE, "edge_lts.h"), "rb") as f:
        h.update(f.read())
    for obj in hip_names:
        with open(os.path.join(BUILD, obj), "rb") as f:
            h.update(f.read())
    key = h.hexdigest()[:16]
    lib = os.path.join(san, f"libedge_lts_san_{key}.so")
    gen = os.path.join(san, f"gen_refmats_san_{key}")
    if not (os.path.exists(lib) and os.path.exists(gen)):
        cxx = ["g++", "-std=c++17", "-O1", "-g", "-fPIC"] + SANITIZE
        inc = ["-I", CSRC, "-I", INCLUDE]
        _run(cxx + ["-o", gen + ".tmp", os.path.join(CSRC, "gen_refmats.cpp"), os.path.join(CSRC, "basis.cpp")])

        def unit(src):
            obj = os.path.join(san, os.path.splitext(src)[0] + "_san.o")
            extra = ["-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"] if src == "host.cpp" else []
            _run(cxx + extra + inc + ["-c", os.path.join(CSRC, src), "-o", obj])
            return obj

        with ThreadPoolExecutor(max_workers=2) as ex:
            objs = list(ex.map(unit, ["host.cpp", "basis.cpp"]))
        hip_objs = [os.path.join(BUILD, o) for o in hip_names]
        _run(["g++", "-shared"] + SANITIZE + ["-o", lib + ".tmp"] + objs + hip_objs +
             ["-L", "/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
        os.replace(gen + ".tmp", gen)
        os.replace(lib + ".tmp", lib)
        for name in os.listdir(san):   # builds of earlier sources
            if name.startswith(("libedge_lts_san_", "gen_refmats_san_")) and key not in name:
                os.remove(os.path.join(san, name))
    return {"lib": lib, "gen": gen, "runtime": sanitizer_runtime()}


if __name__ == "__main__":
    build(verbose=True)
