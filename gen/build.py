"""Build the input generator's C helper (``gen/libgenasm.so``) with gcc.

Input generation only (assembly of element contributions); no solver
arithmetic.  Contractions into fused multiply-adds are disabled so the sums
round exactly as the numpy assembly does.
"""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libgenasm.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "assemble.c")
    tmp = SO + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-o", tmp, src]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, SO)
    return SO


def ensure_built() -> str:
    src = os.path.join(HERE, "assemble.c")
    if not os.path.exists(SO) or os.path.getmtime(SO) < os.path.getmtime(src):
        build()
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
