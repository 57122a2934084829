"""Builds the HIP library in-tree: paper_2312_07874_amd/libesdsem.so (gfx950).

    python paper_2312_07874_amd/build.py [-v]

(run it as a script: importing the package itself requires the built library)

Host setup is plain C++ (g++), the C ABI and the kernels go through hipcc.
Object files live in paper_2312_07874_amd/_build/.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libesdsem.so")
INCLUDE = os.path.join(ROOT, "include")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", INCLUDE, "-I", CSRC, "-Wno-unused-result"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd[:3])} ...")
    if verbose and r.stderr.strip():
        sys.stderr.write(r.stderr)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = [
        ["g++", "-O2", "-std=c++17", "-fPIC", "-pthread", "-I", INCLUDE, "-I", CSRC, "-c",
         os.path.join(CSRC, "host_setup.cpp"), "-o", os.path.join(BUILD, "host_setup.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "api.cpp"), "-o", os.path.join(BUILD, "api.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "kernels.hip"), "-o", os.path.join(BUILD, "kernels.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "adjoint.hip"), "-o", os.path.join(BUILD, "adjoint.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "diagnostics.hip"), "-o", os.path.join(BUILD, "diagnostics.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "batch.hip"), "-o", os.path.join(BUILD, "batch.o")],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "scratch.hip"), "-o", os.path.join(BUILD, "scratch.o")],
    ]
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        list(ex.map(lambda c: _run(c, verbose), jobs))
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp,
          os.path.join(BUILD, "host_setup.o"), os.path.join(BUILD, "api.o"), os.path.join(BUILD, "kernels.o"),
          os.path.join(BUILD, "adjoint.o"), os.path.join(BUILD, "diagnostics.o"),
          os.path.join(BUILD, "batch.o"), os.path.join(BUILD, "scratch.o"), "-pthread"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
