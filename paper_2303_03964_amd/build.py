"""Compile the HIP sources of the library into libtfdp.so for gfx950.

Run as ``python -m paper_2303_03964_amd.build`` (or via ``build()`` in the
repository's entry module). Always recompiles.
"""
from __future__ import annotations

import concurrent.futures
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libtfdp.so")
ARCH = os.environ.get("TFDP_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    f"--offload-arch={ARCH}",
    # keep the compiler from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fuse multiply-adds only inside one source expression: the same code
    # then rounds the same way in every kernel that inlines it (the batched
    # kernels reproduce the per-graph ones bit for bit)
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build_library(verbose: bool = True) -> str:
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    objdir = os.path.join(ROOT, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.basename(src) + ".o") for src in srcs]
    cmds = [[hipcc(), *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj] for src, obj in zip(srcs, objs)]
    if verbose:
        for cmd in cmds:
            print(" ".join(cmd), flush=True)
    # one compiler process per translation unit, at most four at a time
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(4, len(cmds))) as ex:
        for res in ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds):
            if res.stderr:
                sys.stderr.write(res.stderr)
            if res.returncode != 0:
                raise subprocess.CalledProcessError(res.returncode, res.args, res.stdout, res.stderr)
    tmp = LIB + ".tmp"
    # every symbol resolved at link time: a missing definition fails the build,
    # not the first call
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,--no-undefined", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build_library(verbose="-q" not in sys.argv)
