"""Build the gfx950 shared library in-tree with hipcc.

    python -m paper_2510_23221_amd.build

Every HIP source is compiled for gfx950 only, with packed FP32 instructions
disabled, to its own object (in parallel, under ``_build/``) and linked into
``paper_2510_23221_amd/libblockoa.so``.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libblockoa.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["capi.hip", "stencil.hip", "combine.hip", "blockcg.hip", "cg.hip", "nn.hip", "noalloc.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the ROCm toolchain is required to build the library")


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build_library(force: bool = True, verbose: bool = False) -> str:
    srcs = sources()
    deps = srcs + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".hpp")]
    deps.append(os.path.join(os.path.dirname(HERE), "include", "blockoa.h"))
    if not force and os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(d) for d in deps):
        return LIB
    flags = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]
    os.makedirs(OBJDIR, exist_ok=True)
    tag = os.getpid()

    def compile_one(src):
        obj = os.path.join(OBJDIR, os.path.basename(src) + f".{tag}.o")
        cmd = [hipcc(), *flags, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError(f"hipcc failed on {os.path.basename(src)} with status {res.returncode}")
        return obj

    with ThreadPoolExecutor(max_workers=min(len(srcs), 8)) as pool:
        objs = list(pool.map(compile_one, srcs))
    tmp = LIB + f".tmp{tag}"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-fPIC", "-shared", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    for o in objs:
        os.remove(o)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc link failed with status {res.returncode}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(force=True, verbose=True))
