"""Build libvtm.so (HIP for gfx950 + host C++) in-tree.

hipcc compiles the device code and the HIP-runtime host code; g++ compiles the
pure host C++ (partitioner, symbolic analysis).  Every build recompiles.
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libvtm.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = os.environ.get("VTM_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-x", "hip",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics", "-Wall", "-Wno-unused-result", f"-I{INC}", f"-I{CSRC}"]
CXX_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fopenmp", "-Wall", f"-I{INC}", f"-I{CSRC}",
             f"-I{ROCM}/include", "-D__HIP_PLATFORM_AMD__"]

HIP_SRCS = ["kernels.hip", "mlp.hip", "capi.cpp", "zmodel.cpp"]
CXX_SRCS = ["partition.cpp", "symbolic.cpp", "features.cpp"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r.stderr


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for s in HIP_SRCS:
        o = os.path.join(BUILD, s + ".o")
        jobs.append([os.path.join(ROCM, "bin", "hipcc")] + HIP_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
    for s in CXX_SRCS:
        o = os.path.join(BUILD, s + ".o")
        jobs.append(["g++"] + CXX_FLAGS + ["-c", os.path.join(CSRC, s), "-o", o])
    with ThreadPoolExecutor(max_workers=4) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    objs = [os.path.join(BUILD, s + ".o") for s in HIP_SRCS + CXX_SRCS]
    tmp = LIB + ".tmp"
    _run(["g++", "-shared", "-fPIC", "-fopenmp", "-o", tmp] + objs +
         [f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
