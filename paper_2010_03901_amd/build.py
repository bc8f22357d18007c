"""Build libfc2d.so (HIP kernels for gfx950 + host plan code) in-tree.

usage: python -m paper_2010_03901_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import time
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libfc2d.so")
BUILD = os.path.join(ROOT, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HOST_SRC = ["plan.cpp", "matching_host.cpp", "fcgram_quad.cpp", "batch.cpp", "poisson.cpp", "workspace.cpp", "ffsolve.cpp"]
HIP_SRC = ["kernels_plan.hip", "kernels_extend.hip", "kernels_fft.hip", "kernels_mlp.hip", "kernels_poisson.hip",
           "kernels_ffsolve.hip"]

HIPCC_FLAGS = [
    "-O3", "-fPIC", "-std=c++17", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]
GXX_FLAGS = [
    "-O2", "-fPIC", "-std=gnu++17", "-ffp-contract=off", "-fno-builtin-sin", "-fno-builtin-cos",
    "-fopenmp", "-Wno-unknown-pragmas",
    "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"), "-Wall", "-Wno-unused-function",
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout)
        raise RuntimeError("build step failed: " + os.path.basename(cmd[-1]))
    return r.stdout


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    gxx = shutil.which("g++") or "g++"
    jobs = [[gxx] + GXX_FLAGS + ["-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, src + ".o")]
            for src in HOST_SRC]
    jobs += [[hipcc] + HIPCC_FLAGS + ["-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, src + ".o")]
             for src in HIP_SRC]
    objs = [j[-1] for j in jobs]
    t0 = time.time()
    # the translation units are independent: compile them side by side
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1, 8)) as ex:
        list(ex.map(_run, jobs))
    tmp = OUT + ".tmp"
    _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs +
         ["-lquadmath", "-lgomp", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    os.replace(tmp, OUT)
    if verbose:
        print("built %s in %.1f s" % (OUT, time.time() - t0))
    return OUT


if __name__ == "__main__":
    build(verbose=True)
