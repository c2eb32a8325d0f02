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


# host-side AddressSanitizer and UBSan (each -fsanitize= behind -Xarch_host: the
# device code is compiled without them)
SAN_HOST_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
HOST_SOURCES = ["rod_lib.cpp", "surrogate.cpp"]   # no device code


def build_sanitized(outdir: str) -> str:
    """librod with AddressSanitizer and UBSan in the host runtime (descriptor
    validation, input gathering and checks, tile packing, derivation of the
    per-slot constants, the surrogate's host logic), linked with the regular
    build's kernel objects.  Returns the library's path; it runs in a process
    that has clang's ASan runtime (asan_runtime()) preloaded."""
    default = os.path.join(HERE, "_build", "default")
    if not all(os.path.exists(os.path.join(default, os.path.splitext(s)[0] + ".o")) for s in SOURCES):
        build()
    os.makedirs(outdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        base = os.path.splitext(src)[0] + ".o"
        if src not in HOST_SOURCES:
            objs.append(os.path.join(default, base))
            continue
        obj = os.path.join(outdir, base)
        cmd = [hipcc(), f"--offload-arch={ARCH}", "-O1", "-g", "-std=c++17", "-fPIC", "-x", "hip",
               "--offload-host-only", *SAN_HOST_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src),
               "-o", obj]
        subprocess.check_call(cmd)
        objs.append(obj)
    out = os.path.join(outdir, "librod_san.so")
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(hipcc())))
    clangxx = os.path.join(rocm, "llvm", "bin", "clang++")
    subprocess.check_call([clangxx, "-shared", "-fsanitize=address,undefined", "-shared-libasan", "-o", out, *objs,
                           "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(rocm, "lib")])
    return out


def asan_runtime() -> str:
    """Path of clang's shared ASan runtime (to preload for build_sanitized's library)."""
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(hipcc())))
    out = subprocess.check_output([os.path.join(rocm, "llvm", "bin", "clang++"),
                                   "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()
    if not os.path.isabs(out):
        import glob
        cands = glob.glob(os.path.join(rocm, "llvm", "lib", "clang", "*", "lib", "linux", "libclang_rt.asan-x86_64.so"))
        if not cands:
            raise RuntimeError("clang's shared ASan runtime not found")
        out = cands[0]
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
