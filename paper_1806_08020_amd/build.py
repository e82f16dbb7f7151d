"""Build libppa.so (hand-written HIP for gfx950) in-tree with hipcc, and the
benchmark's bandwidth reference kernels (libppa_bwprobe.so, no part of the
solver).

Usage: ``python -m paper_1806_08020_amd.build`` (or ``build()`` from Python).
Every call recompiles all sources.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libppa.so")
SOURCES = ["spmv.hip", "blas.hip", "dense.cpp", "ritz.cpp", "poly.cpp", "eigs.cpp", "batch.hip", "api.cpp"]
PROBE_SRC = "bwprobe.hip"
PROBE_LIB = os.path.join(HERE, "libppa_bwprobe.so")
ARCH = "gfx950"

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep packed FP32 ops out of generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-function",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, build_dir: str = BUILD, defines=()) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *COMMON, *[f"-D{d}" for d in defines], "-x", "hip", "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def _link(objs, out: str) -> None:
    tmp = out + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)


def build(verbose: bool = False, out: str = LIB, build_dir: str = BUILD, defines=()) -> str:
    """Compile all sources and link `out`.  `defines` override tuning
    constants (PPA_SPMV_CHUNK, PPA_SPMV_BS, PPA_CGS_RPT, PPA_CGS_CT).  The
    default build also links libppa_bwprobe.so."""
    os.makedirs(build_dir, exist_ok=True)
    srcs = SOURCES + ([PROBE_SRC] if out == LIB else [])
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda f: _compile(f, build_dir, defines), srcs))
    _link(objs[:len(SOURCES)], out)
    if verbose:
        print("built", out)
    if out == LIB:
        _link(objs[len(SOURCES):], PROBE_LIB)
        if verbose:
            print("built", PROBE_LIB)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
