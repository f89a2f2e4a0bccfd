"""Build the oracle's C library (``oracle/liboracle.so``) with gcc.

Test infrastructure: the library built here is loaded only by the test
suite, the smoke check and the CPU-baseline leg of the benchmark.
"""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "oracle.c")
    tmp = SO + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, SO)
    return SO


def ensure_built() -> str:
    src = os.path.join(HERE, "oracle.c")
    if not os.path.exists(SO) or os.path.getmtime(SO) < os.path.getmtime(src):
        build()
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
