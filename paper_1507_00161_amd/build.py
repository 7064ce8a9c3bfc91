"""Build libdmrg_mi355x.so in-tree with hipcc for gfx950.

    python -m paper_1507_00161_amd.build        (or python paper_1507_00161_amd/build.py)

Every source is compiled on each call (hipcc cross-compiles without a GPU).
Packed-FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libdmrg_mi355x.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-Wall", "-pthread"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False) -> str:
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    dev_obj = os.path.join(objdir, "device.o")
    _run([hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, "device.hip"), "-o", dev_obj])
    objs.append(dev_obj)
    for src in ("engine.cpp", "capi.cpp", "entropy.cpp", "batch.cpp"):
        obj = os.path.join(objdir, src.replace(".cpp", ".o"))
        _run(["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    tmp = OUT + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp,
          f"-L{ROCM}/lib", "-lrocsolver", "-lrocblas", "-lpthread", f"-Wl,-rpath,{ROCM}/lib"])
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
