"""Build the CPU oracle (test infrastructure) with g++: oracle/liborc.so.

Plain FP64: -O2, no fast-math, no FMA contraction, so the oracle evaluates the
paper's expressions in IEEE double in the order written.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pf_oracle.cpp")
OUT = os.path.join(HERE, "liborc.so")


OUT_OMP = os.path.join(HERE, "liborc_omp.so")


def build(verbose: bool = False) -> str:
    """liborc.so (single thread) and liborc_omp.so (the same source with its
    OpenMP cell loops enabled, used only to time the oracle on all host cores)."""
    base = ["g++", "-O2", "-std=c++17", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
            "-Wextra"]
    for out, extra in ((OUT, ["-Wno-unknown-pragmas"]), (OUT_OMP, ["-fopenmp"])):
        cmd = base + extra + ["-o", out + ".tmp", SRC]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
