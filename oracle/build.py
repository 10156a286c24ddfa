"""Build the FP64 CPU oracle library (test infrastructure) with gcc.

Flags: -O2, no fast-math, -ffp-contract=off so that no multiply-add is fused
behind the source's back.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# The same source with its OpenMP loop pragmas enabled: only the CPU-baseline
# leg of the benchmark loads it (to time the oracle on all host cores).
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def _build_one(out: str, extra: list, verbose: bool) -> str:
    tmp = out + f".tmp{os.getpid()}"
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unknown-pragmas", *extra, "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    """Builds the reference oracle (sequential, used by the tests) and its
    OpenMP timing build; returns the reference library's path."""
    _build_one(LIB, [], verbose)
    _build_one(LIB_OMP, ["-fopenmp"], verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
