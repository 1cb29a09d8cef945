"""Build libqsmg.so for gfx950 in-tree (hipcc for the HIP sources, g++ for host code)."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libqsmg.so")
BUILD = os.path.join(PKG, "_build")

HIP_SOURCES = ["kernels_mg.hip", "kernels_sweep.hip", "kernels_resid.hip", "kernels_stz.hip", "api.hip"]
HOST_SOURCES = ["hierarchy.cpp"]
# Packed FP32 instructions are disabled for all device code.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return r


def build_library(verbose: bool = False) -> str:
    """Compile every source (in parallel, one process per file) and link."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    jobs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append((obj, ["g++", "-O3", "-std=c++17", "-fPIC", "-Wall", "-c",
                           os.path.join(CSRC, src), "-I", INCLUDE, "-o", obj]))
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append((obj, [hipcc] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-I", INCLUDE,
                                                 "-I", CSRC, "-o", obj]))
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(lambda j: _run(j[1]), jobs))
    if verbose:
        for r in results:
            if r.stderr:
                print(r.stderr)
    objs = [j[0] for j in jobs]
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
