"""Build librod.so (HIP for gfx950) in-tree with hipcc.

Every HIP translation unit is compiled with packed-FP32 instruction
selection turned off and with FMA contraction limited to single source
expressions.  Run as ``python -m paper_2605_13766_amd.build``.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "librod.so")

ARCH = "gfx950"
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # contract a*b+c only inside one source expression: the same FMAs in every
    # tile-width instantiation, so results do not depend on the launch shape
    "-ffp-contract=on",
    "-Wno-unused-command-line-argument",
]

SOURCES = ["rod_lib.cpp", "rod_kernels.hip", "contact_kernels.hip", "noalloc.hip", "surrogate.cpp", "mlp_kernels.hip", "mlp_infer.hip", "surrogate_kernels.hip"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, defines=(), out: str = LIB) -> str:
    """Compile every source and link librod.so (or `out`); returns its path.
    `defines` are extra -D macros (tuning variants)."""
    objs = []
    bdir = os.path.join(HERE, "_build", "x".join(defines).replace("=", "") or "default")
    os.makedirs(bdir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), *HIP_FLAGS, *[f"-D{d}" for d in defines], "-x", "hip", "-I", INCLUDE, "-I", CSRC, "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
