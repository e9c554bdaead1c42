"""Build the gfx950 shared library ``libfcsdnn.so`` in this package directory.

Host-only C++ that needs quad precision (the FC-Gram builder, grids and
connectivity) is compiled with g++; the HIP kernels and the C ABI with hipcc
for gfx950.  Usage: ``python -m paper_2506_19370_amd.build`` (or through
``__graft_entry__.build()``).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libfcsdnn.so")
BUILD = os.path.join(HERE, "_build")

GXX_SOURCES = ["fc_builder.cpp", "geometry.cpp"]
HIP_SOURCES = ["gemm.hip", "stage_kernels.hip", "window_kernels.hip", "sdnn_train.hip", "api.cpp", "aux_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
GXX_FLAGS = ["-O2", "-std=gnu++17", "-fext-numeric-literals", "-fPIC", "-pthread"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed: " + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for src in GXX_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append(["g++", *GXX_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        jobs.append([HIPCC, *HIP_FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for out in ex.map(_run, jobs):
            if verbose and out.strip():
                print(out)
    objs = [os.path.join(BUILD, s + ".o") for s in GXX_SOURCES + HIP_SOURCES]
    tmp = OUT + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-lquadmath", "-lpthread"])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
