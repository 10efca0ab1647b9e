"""Build ``libcavity.so`` (HIP kernels + host runtime + C ABI) for gfx950.

Run ``python -m paper_0809_3098_amd.build``.  hipcc cross-compiles for the
MI355X's gfx950 target; no GPU is needed to build.  The library is written
in-tree next to this file so that it travels with the source tree.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcavity.so")
SOURCES = ["cavity_kernels.hip", "cavity_runtime.cpp"]
ARCH = "gfx950"

# Packed FP32 instructions are disabled: the compiler may not form them from
# ordinary float code.
COMMON_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; ROCm is required to build libcavity.so")
    return exe


def build(verbose: bool = False) -> str:
    """Compile every source and link ``libcavity.so``; returns its path."""
    cc = hipcc()
    objdir = os.path.join(ROOT, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [cc, *COMMON_FLAGS, "-I", os.path.join(ROOT, "include"), *lang, "-c",
               os.path.join(CSRC, src), "-o", obj]
        _run(cmd, verbose)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([cc, "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    build_demo(verbose)
    return LIB


DEMO_SRC = os.path.join(HERE, "examples", "cavity_step_demo.c")
DEMO = os.path.join(HERE, "examples", "cavity_step_demo")


def build_demo(verbose: bool = False) -> str:
    """The plain C caller of the ABI, compiled as C99 by the host C compiler."""
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        raise RuntimeError("no C compiler for the C example")
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(hipcc())))
    _run([cc, "-std=c99", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__",
          "-I", os.path.join(rocm, "include"), "-I", os.path.join(ROOT, "include"), DEMO_SRC,
          "-o", DEMO, "-L", HERE, "-lcavity", "-L", os.path.join(rocm, "lib"), "-lamdhip64",
          "-Wl,-rpath,$ORIGIN/..", "-Wl,-rpath," + os.path.join(rocm, "lib")], verbose)
    return DEMO


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in res.stdout.splitlines()
                    if "packed-fp32-ops" not in l and "not a recognized feature" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"build step failed ({res.returncode}): {' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
