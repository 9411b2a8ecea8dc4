"""Builds libbatchode.so (HIP for gfx950) in-tree.

Every source under csrc/ is compiled with hipcc for gfx950 only and linked
into paper_2210_12375_amd/libbatchode.so.  Packed FP32 instructions are
disabled for all device code (the feature flag goes to the device pass; the
host pass ignores it with a warning).
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbatchode.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
         "-Wno-unused-command-line-argument"]


def sources():
    return sorted(f for f in os.listdir(CSRC)
                  if f.endswith(".hip") or f.endswith(".cpp"))


def _compile(src, verbose):
    obj = os.path.join(OBJ, src + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines()
                     if "packed-fp32-ops" not in l and l.strip()
                     and "warning generated" not in l)
    if verbose and warn:
        print(warn, flush=True)
    return obj


CEIL_SRC = os.path.join(HERE, "ceilings", "ceilings.hip")
CEIL_LIB = os.path.join(HERE, "libceilings.so")


def build_ceilings(verbose: bool = False) -> str:
    """The measurement-only ceilings library (bench.py's achievable peaks)."""
    cmd = [HIPCC] + FLAGS + ["-shared", CEIL_SRC, "-o", CEIL_LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on ceilings.hip:\n{r.stdout}\n"
                           f"{r.stderr}")
    os.replace(CEIL_LIB + ".tmp", CEIL_LIB)
    return CEIL_LIB


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=max(1, min(jobs, len(srcs)))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(LIB + ".tmp", LIB)
    build_ceilings(verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
