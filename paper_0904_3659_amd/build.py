"""Build libnbody.so (HIP, gfx950) in-tree with hipcc.

Run as ``python -m paper_0904_3659_amd.build``; ``__graft_entry__.build()``
calls :func:`build`.
"""

from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBRARY = os.path.join(HERE, "libnbody.so")
ARCH = "gfx950"

HIPFLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # Packed FP32 (v_pk_*_f32) generation stays off; every float op is a
    # plain VALU instruction.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast", "-Wall", "-Wno-unused-function",
]


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    tmp = LIBRARY + ".tmp"
    cmd = ["hipcc", *HIPFLAGS, *(extra or []), *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIBRARY)
    return LIBRARY


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
