"""Compile the FP64 reference library (plain C, OpenMP, no fast-math).

TEST INFRASTRUCTURE ONLY.  Run as ``python -m oracle.build`` or through
``__graft_entry__.build()``.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "nbody_oracle.c")
LIBRARY = os.path.join(HERE, "libnbody_oracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
          "-fno-fast-math", "-ffp-contract=off", "-fno-math-errno"]


def build(verbose: bool = False) -> str:
    tmp = LIBRARY + ".tmp"
    cmd = ["gcc", *CFLAGS, SOURCE, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIBRARY)
    return LIBRARY


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
