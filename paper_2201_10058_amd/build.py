"""Build libgenga.so (gfx950) in-tree with hipcc.

Every HIP source under csrc/ is compiled for gfx950 and linked into
paper_2201_10058_amd/libgenga.so.  Packed FP32 instructions are disabled, and
floating-point contraction is off: every fused multiply-add in the kernels is
an explicit __builtin_fma.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libgenga.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared", "-mcode-object-version=5",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def assemble(out_dir: str, verbose: bool = False) -> list:
    """Write the gfx950 assembly of every source to out_dir (for inspection)."""
    os.makedirs(out_dir, exist_ok=True)
    outs = []
    for src in sources():
        out = os.path.join(out_dir, os.path.basename(src).replace(".hip", ".s"))
        cmd = [HIPCC, *[f for f in FLAGS if f not in ("-shared", "-fPIC")], "--cuda-device-only",
               "-S", src, "-o", out]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        outs.append(out)
    return outs


if __name__ == "__main__":
    if "-S" in sys.argv:
        # python build.py -S OUT_DIR: the assembly of every source into OUT_DIR
        k = sys.argv.index("-S")
        if k + 1 >= len(sys.argv):
            sys.exit("usage: build.py -S OUT_DIR")
        print(assemble(sys.argv[k + 1], verbose=True))
    else:
        print(build(verbose="-v" in sys.argv))
