"""Builds librsc.so in-tree: host C++ with g++, the gfx950 kernels with hipcc.

Usage: python -m paper_1507_05593_amd.build  (or build() from Python).
Every call recompiles every source.
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "librsc.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

HOST_SOURCES = ["symbolic.cpp", "runtime.cpp", "spectral.cpp", "api.cpp"]
HIP_SOURCES = ["kernels_dense.hip", "kernels_pcg.hip", "kernels_gemm.hip", "kernels_spectral.hip"]
COMMON = ["-std=c++17", "-O3", "-fPIC", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
HIP_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError("build step failed: " + " ".join(cmd) + "\n" + p.stdout)
    return p.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    jobs = []
    for s in HOST_SOURCES:
        o = os.path.join(OUT, s + ".o")
        jobs.append(["g++"] + COMMON + ["-I" + os.path.join(ROCM, "include"), "-D__HIP_PLATFORM_AMD__",
                                        "-c", os.path.join(CSRC, s), "-o", o])
    for s in HIP_SOURCES:
        o = os.path.join(OUT, s + ".o")
        jobs.append([HIPCC] + COMMON + HIP_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        logs = list(ex.map(_run, jobs))
    objs = [j[-1] for j in jobs]
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "--offload-arch=gfx950", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    if verbose:
        for l in logs:
            if l.strip():
                print(l)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
