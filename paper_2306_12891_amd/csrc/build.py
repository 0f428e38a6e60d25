"""Builds libdgmi.so (HIP, gfx950) in-tree: one kernel object per polynomial
degree, compiled in parallel, plus the host object, linked with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
OUT = os.path.join(PKG, "libdgmi.so")
BUILD = os.path.join(ROOT, "_build")
DEGREES = range(1, 8)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wno-unused-result",
         # keep the compiler from emitting packed FP32 arithmetic
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", HERE]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("compile failed: " + " ".join(cmd[-3:]))
    return r.stdout


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compiles the committed kernel and host sources and links the library."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    kernel_source = os.path.join(HERE, "dg_kernels.hip")
    cmds = []
    for n in DEGREES:
        obj = os.path.join(BUILD, f"dg_kernels_N{n}.o")
        cmds.append([HIPCC, *FLAGS, f"-DDG_N={n}", "-c", kernel_source, "-o", obj])
    host_obj = os.path.join(BUILD, "dg_host.o")
    cmds.append([HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(HERE, "dg_host.cpp"), "-o", host_obj])
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    objs = [c[-1] for c in cmds]
    tmp = OUT + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
