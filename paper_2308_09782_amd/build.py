"""Compile the gfx950 shared library (libvgtb.so) in-tree with hipcc.

Each HIP source is compiled to its own object (in parallel, under
paper_2308_09782_amd/_build/) so that a file can carry its own code-generation
flags, then the objects are linked against rocSOLVER/rocBLAS.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libvgtb.so")
OBJDIR = os.path.join(PKG, "_build")
ARCH = "gfx950"

# Per-file flags.  kernels.hip: keep the FP64 matrix-core accumulators of the
# sparse product in ordinary VGPRs (its epilogue does vector arithmetic on
# them; in AGPRs they would all be copied out at once and cut occupancy).
FILE_FLAGS = {"kernels.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def sources() -> list:
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))


def compile_command(src: str, obj: str) -> list:
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-c", "-Wall",
            # keep the compiler from forming packed-FP32 instructions
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            *FILE_FLAGS.get(os.path.basename(src), []),
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"), src, "-o", obj]


def link_command(objs: list, out: str = LIB) -> list:
    return [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-L/opt/rocm/lib",
            "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib", "-o", out]


def command(out: str = LIB) -> list:
    """The compile commands (one per source) followed by the link command."""
    srcs = sources()
    objs = [os.path.join(OBJDIR, os.path.basename(s) + ".o") for s in srcs]
    return [compile_command(s, o) for s, o in zip(srcs, objs)] + [link_command(objs, out)]


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    tmp = LIB + ".tmp"
    cmds = command(tmp)
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    with ThreadPoolExecutor(max_workers=min(len(cmds) - 1, 8)) as ex:
        for f in [ex.submit(subprocess.run, c, check=True) for c in cmds[:-1]]:
            f.result()
    subprocess.run(cmds[-1], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
