"""Build the FP64 CPU oracle library (test infrastructure only).

gcc, -O3, OpenMP, no FMA contraction and no fast-math, generic x86-64 code
so the library built here also runs on other hosts.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sph_oracle.c")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libsph_oracle.so")


def build(verbose: bool = False, src: str = SRC, out: str = LIB) -> str:
    """Compile ``src`` (default: the oracle) into the shared library ``out``."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp"
    cmd = ["gcc", "-O3", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wno-unused-function", src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
