"""Builds the HIP library ``libhho_pmg.so`` in-tree for gfx950.

Host-only C++ (mesh import, quadrature, bases, local HHO operators) is built
with g++; the HIP translation units (kernels, setup/solve orchestration, C ABI)
with hipcc for gfx950.  Usage: ``python -m paper_2009_13840_amd.build``.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhho_pmg.so")
BUILD = os.path.join(os.path.dirname(HERE), "_build")

HOST_SRC = ["host_mesh.cpp", "host_local.cpp", "amg_host.cpp", "nd_host.cpp"]
HIP_SRC = ["k_setup.hip", "k_solve.hip", "k_spmv.hip", "k_orth.hip", "k_amg.hip", "k_mlp.hip", "k_local.hip", "k_ilu.hip", "k_direct.hip", "solver.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("HHO_OFFLOAD_ARCH", "gfx950")
HIP_FLAGS = ["-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_FLAGS = ["-std=c++17", "-O3", "-fPIC", "-pthread", "-Wall", "-Wno-unused-function"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for f in HOST_SRC:
        o = os.path.join(BUILD, f + ".o")
        jobs.append(["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, f), "-o", o])
    for f in HIP_SRC:
        o = os.path.join(BUILD, f + ".o")
        jobs.append([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, f), "-o", o])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout, r.stderr)
    objs = [os.path.join(BUILD, f + ".o") for f in HOST_SRC + HIP_SRC]
    tmp = OUT + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-pthread"])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
