"""Compile the CPU oracle (plain C, gcc) into ``oracle/libcns_oracle.so``.

Test infrastructure: the oracle is loaded only by the tests, the smoke check
and the benchmark's CPU-baseline leg.  Built with ``-O2 -ffp-contract=off``
(no fused multiply-add, so every product is rounded as written) and OpenMP
for the independent per-point loops.  No ``-march=native``: the library is
also run on other hosts.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cns_oracle.c")
LIB = os.path.join(HERE, "libcns_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
