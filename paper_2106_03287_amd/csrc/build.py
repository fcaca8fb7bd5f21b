"""Build libstein_icp.so for gfx950 with hipcc (in-tree, next to the package)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
INCLUDE = os.path.join(ROOT, "include")
# (source, extra flags): the BF16 screen is built with IEEE mode off
SOURCES = [
    (os.path.join(HERE, "stein_icp.hip"), []),
    (os.path.join(HERE, "nn_bf16.hip"), ["-fno-honor-nans", "-mno-amdgpu-ieee"]),
    (os.path.join(HERE, "proposal.hip"), []),
    (os.path.join(HERE, "peaks.hip"), []),
]
OUT = os.path.join(PKG, "libstein_icp.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(out: str = OUT, extra=()) -> str:
    objs = []
    for src, flags in SOURCES:
        obj = os.path.join(os.path.dirname(out), "_" + os.path.basename(src) + ".o")
        cflags = [f for f in FLAGS if f != "-shared"]
        subprocess.check_call([HIPCC, *cflags, *flags, *extra, f"-I{INCLUDE}", f"-I{HERE}", "-c", src, "-o", obj])
        objs.append(obj)
    tmp = out + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    for o in objs:
        os.remove(o)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(extra=sys.argv[1:]))
