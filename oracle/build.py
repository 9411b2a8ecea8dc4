"""Builds the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain C11 with OpenMP over instances; -ffp-contract=off keeps every
multiply-add as written, so the oracle rounds the way its source reads.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["tableau.c", "rhs.c", "solve.c", "adjoint.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC",
           "-Wall", "-Wextra", "-shared", "-o", LIB + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def needs_build() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = SOURCES + ["oracle.h"]
    return any(os.path.getmtime(os.path.join(HERE, s)) > t for s in deps)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
