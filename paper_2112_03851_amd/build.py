"""Build the HIP library libsos.so in-tree for gfx950 with hipcc.

The sources compile to objects in parallel (the fused CG kernel once per
number of x-y columns per thread, 1 to 4) and are linked into one shared
library next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsos.so")
CSRC = os.path.join(HERE, "csrc")
OBJDIR = os.path.join(HERE, "_build")
ARCH = "gfx950"
# (source, extra defines, object name)
UNITS = [("sos_kernels.hip", [], "sos_kernels.o"),
         ("sos_api.hip", [], "sos_api.o"),
         ("sos_cmaes.cpp", [], "sos_cmaes.o")] + \
        [("sos_fused.hip", [f"-DSOS_FUSED_CPT={c}"], f"sos_fused_c{c}.o") for c in (1, 2, 3, 4)]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


def _flags():
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            # packed FP32 instructions are kept out of the generated code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include")]


def _compile(unit, verbose):
    src, defs, obj = unit
    cmd = [hipcc(), *_flags(), *defs, "-c", os.path.join(CSRC, src), "-o", os.path.join(OBJDIR, obj)]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    return cmd, res


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source and link libsos.so (always rebuilds)."""
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(len(UNITS), max(1, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda u: _compile(u, verbose), UNITS))
    for cmd, res in results:
        if res.returncode != 0:
            sys.stderr.write(" ".join(cmd) + "\n" + res.stdout + res.stderr)
            raise RuntimeError("hipcc failed building libsos.so")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *[os.path.join(OBJDIR, u[2]) for u in UNITS],
           # roctx ranges around the outer iterations (rocprofv3 --marker-trace)
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libsos.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
