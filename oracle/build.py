"""Build the C oracle into oracle/libgenga_oracle.so with gcc.

TEST INFRASTRUCTURE ONLY (see genga_oracle.c).  Contraction is disabled so
that every product and sum is a separately rounded binary64 operation; the
target is x86-64-v3 so the library also runs on the GPU host's CPU.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "genga_oracle.c")
LIB = os.path.join(HERE, "libgenga_oracle.so")

CFLAGS = ["-O2", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
