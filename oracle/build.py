"""Builds the CPU oracle (test infrastructure) into oracle/libcg_oracle.so.

Plain gcc, -O2 with floating-point contraction off and no fast-math, so that
every arithmetic operation in cg_oracle.c is one correctly rounded IEEE
operation; cg_oracle_fixed.c (the fixed-point variant) is integer code.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = [os.path.join(HERE, f) for f in ("cg_oracle.c", "cg_oracle_fixed.c")]
LIB = os.path.join(HERE, "libcg_oracle.so")
# the all-core timing build of the same sources (CPU baseline only)
LIB_OMP = os.path.join(HERE, "libcg_oracle_omp.so")


def stale(omp: bool = False) -> bool:
    """True when the library is missing or older than a source."""
    lib = LIB_OMP if omp else LIB
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    return any(os.path.getmtime(f) > t for f in SOURCES)


def build(verbose: bool = False, omp: bool = False) -> str:
    lib = LIB_OMP if omp else LIB
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           "-Wno-unknown-pragmas", "-fPIC", "-shared"] + (["-fopenmp"] if omp else []) + \
          ["-o", tmp] + SOURCES + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def build_all(verbose: bool = False):
    build(verbose)
    build(verbose, omp=True)


if __name__ == "__main__":
    build_all(verbose="-v" in sys.argv)
