"""Builds the gfx950 multisplit library in-tree with hipcc.

The library is the product: csrc/*.hip and csrc/*.hpp compiled for
--offload-arch=gfx950 into paper_1701_01189_amd/libmultisplit.so.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmultisplit.so")
SRCS = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
OBJDIR = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed fp32 instructions stay off in every HIP build of this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*"))) + [
        os.path.join(ROOT, "include", "multisplit.h")]


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in sources())


def build(force: bool = True, verbose: bool = False) -> str:
    """Compiles the library (always when force, else only when stale)."""
    if not force and not stale():
        return LIB
    os.makedirs(OBJDIR, exist_ok=True)
    objs, procs = [], []
    for src in SRCS:
        obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
        cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    failed = [cmd for p, cmd in procs if p.wait() != 0]
    if failed:
        raise RuntimeError("hipcc failed: %s" % " ".join(failed[0]))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs +
                          ["-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force=True, verbose=True)
    print(LIB)
