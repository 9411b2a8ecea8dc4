"""Builds the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain C11 with OpenMP over instances; -ffp-contract=off keeps every
multiply-add as written, so the oracle rounds the way its source reads.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["tableau.c", "rhs.c", "solve.c", "joint.c", "adjoint.c",
           "cadjoint.c"]
LIB = os.path.join(HERE, "liboracle.so")
# The same source with every a*b+c contracted into a fused multiply-add.  It
# is not a second oracle: the tests use it only to find instances whose step
# counts change under a 1-ulp change of rounding (see tests/gpu_helpers.py).
LIB_FMA = os.path.join(HERE, "liboracle_fma.so")


# The same source built with AddressSanitizer and UndefinedBehaviorSanitizer
# (any report aborts), for a CPU test that runs the oracle's entry points
# under them; loaded only by that test, with the sanitizer runtimes
# preloaded.
LIB_SAN = os.path.join(HERE, "liboracle_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer", "-g"]


def _build_one(out, contract, verbose, extra=()):
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", f"-ffp-contract={contract}",
           "-fPIC", "-Wall", "-Wextra", "-shared", "-o", out + ".tmp"]
    cmd[1:1] = list(extra)
    if contract == "fast":
        cmd.insert(3, "-mfma")
    cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)


def build(verbose: bool = False) -> str:
    _build_one(LIB, "off", verbose)
    _build_one(LIB_FMA, "fast", verbose)
    return LIB


def build_sanitized(verbose: bool = False) -> str:
    _build_one(LIB_SAN, "off", verbose, SAN_FLAGS)
    return LIB_SAN


def needs_build() -> bool:
    for lib in (LIB, LIB_FMA):
        if not os.path.exists(lib):
            return True
        t = os.path.getmtime(lib)
        deps = SOURCES + ["oracle.h"]
        if any(os.path.getmtime(os.path.join(HERE, s)) > t for s in deps):
            return True
    return False


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
