"""Builds the HIP library libcg.so (gfx950) in-tree.

hipcc compiles every source for gfx950 only.  Floating-point contraction is
off everywhere (the kernels write every fused multiply-add explicitly) and
packed-FP32 instructions are disabled.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcg.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["cg_kernels.hip", "cg_fixed.hip", "cg_noalloc.hip", "cg_runtime.cpp", "cg_serve.cpp",
           "cg_abi.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]


def _compile(src):
    out = os.path.join(BUILD, src + ".o")
    lang = [] if src.endswith(".hip") else ["-x", "hip"]
    cmd = [HIPCC] + FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, flush=True)
    return LIB


# The serving runtime's concurrency stress (tests/serve_stress.cpp) in a
# host-sanitized build: the host sources of the runtime and the driver are
# instrumented with AddressSanitizer (the flag reaches the host pass only),
# the kernels' objects are the ones build() made.  (Under ThreadSanitizer the
# HIP runtime finds no device: TSan's memory layout leaves no room for the
# GPU's address-space reservations.)
HOST_SOURCES = ["cg_runtime.cpp", "cg_serve.cpp", "cg_abi.cpp"]
ROOT = os.path.dirname(HERE)
STRESS_SRC = os.path.join(ROOT, "tests", "serve_stress.cpp")
STRESS_DIR = os.path.join(ROOT, "tests", "bin")
SANITIZERS = {
    "asan": ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"],
}


def _compile_san(args):
    kind, src = args
    path = src if os.path.isabs(src) else os.path.join(CSRC, src)
    out = os.path.join(BUILD, "%s_%s.o" % (kind, os.path.basename(src)))
    cmd = ([HIPCC] + FLAGS + ["-g", "-x", "hip", "-I", os.path.join(ROOT, "include")] +
           SANITIZERS[kind] + ["-c", path, "-o", out])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return out


def build_stress(verbose: bool = False) -> list:
    """The stress driver tests/bin/serve_stress_asan; needs build() first."""
    os.makedirs(STRESS_DIR, exist_ok=True)
    kernels = [os.path.join(BUILD, s + ".o") for s in SOURCES if s.endswith(".hip")]
    for k in kernels:
        if not os.path.exists(k):
            raise RuntimeError("build() first: %s is missing" % k)
    jobs = [(kind, s) for kind in SANITIZERS for s in HOST_SOURCES + [STRESS_SRC]]
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(_compile_san, jobs))
    out = []
    for kind in SANITIZERS:
        mine = [o for (kd, _), o in zip(jobs, objs) if kd == kind]
        exe = os.path.join(STRESS_DIR, "serve_stress_" + kind)
        cmd = ([HIPCC, "--offload-arch=gfx950"] + SANITIZERS[kind] + ["-o", exe + ".tmp"] +
               mine + kernels + ["-lpthread"])
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
        os.replace(exe + ".tmp", exe)
        out.append(exe)
        if verbose:
            print("built", exe, flush=True)
    return out


if __name__ == "__main__":
    build(verbose=True)
    build_stress(verbose=True)
