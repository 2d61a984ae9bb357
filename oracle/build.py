"""Builds the CPU oracle library (test infrastructure) with gcc.

    python oracle/build.py

Produces oracle/libngd_oracle.so.  Plain -O2, OpenMP, no fast-math and no
floating-point contraction, so every fma in the sources is an explicit call
and every other operation rounds exactly as written.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["ngd_oracle.c", "ngd_cull_ref.c"]
OUT = os.path.join(HERE, "libngd_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           "-Wno-unused-parameter",
           *[os.path.join(HERE, s) for s in SOURCES], "-o", OUT + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
