"""Compile the CPU oracle (plain C, gcc) into ``oracle/libcns_oracle.so``.

``cns_oracle_cs.c`` compiles the oracle's arithmetic a second time in complex
numbers for complex-step derivatives; both go into the one library.

Test infrastructure: the oracle is loaded only by the tests, the smoke check
and the benchmark's CPU-baseline leg.  Built with ``-O2 -ffp-contract=off``
(no fused multiply-add, so every product is rounded as written) and OpenMP
for the independent per-point loops.  The in-tree library has no
``-march=native`` (it is also run on other hosts); ``build(native=True, out=...)``
makes a build for the host it runs on, which the benchmark times.  Without
fused multiply-adds and without reassociation the two builds round every
operation alike.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cns_oracle.c")
SRC_CS = os.path.join(HERE, "cns_oracle_cs.c")  # the same arithmetic in complex numbers
LIB = os.path.join(HERE, "libcns_oracle.so")


def build(verbose: bool = False, native: bool = False, out: str | None = None) -> str:
    out = out or LIB
    cmd = ["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unused-parameter"] + (["-march=native"] if native else []) + \
          ["-o", out + ".tmp", SRC, SRC_CS, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
