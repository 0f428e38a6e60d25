"""Address/undefined-behaviour sanitizer build of the library's host side and
its C-ABI argument checks (abi_check.cpp), run on the CPU.

dg_host.cpp is compiled with the sanitizers on its host code only (each
-fsanitize= after -Xarch_host; the GPU code is not instrumented) and linked
with the kernel objects of the regular build (build.py) and the check driver.
Returns (exit status, output) of the driver, run with leak detection off (the
HIP runtime keeps its own allocations until exit)."""
from __future__ import annotations

import os
import subprocess

from . import build as B

SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


def build_and_run(timeout: float = 300.0) -> tuple[int, str]:
    if not all(os.path.exists(os.path.join(B.BUILD, f"dg_kernels_N{n}.o")) for n in B.DEGREES):
        B.build()
    out = os.path.join(B.BUILD, "asan")
    os.makedirs(out, exist_ok=True)
    host = os.path.join(out, "dg_host.o")
    drv = os.path.join(out, "abi_check.o")
    exe = os.path.join(out, "abi_check")
    B._run([B.HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", *SAN,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(B.ROOT, "include"),
            "-I", B.HERE, "-x", "hip", "-c", os.path.join(B.HERE, "dg_host.cpp"), "-o", host], False)
    B._run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-I", os.path.join(B.ROOT, "include"),
            "-c", os.path.join(B.HERE, "abi_check.cpp"), "-o", drv], False)
    objs = [os.path.join(B.BUILD, f"dg_kernels_N{n}.o") for n in B.DEGREES]
    B._run([B.HIPCC, "--offload-arch=gfx950", *SAN, "-o", exe, drv, host, *objs], False)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=timeout)
    return r.returncode, r.stdout


if __name__ == "__main__":
    rc, text = build_and_run()
    print(text)
    raise SystemExit(rc)
