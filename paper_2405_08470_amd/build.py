"""Builds libspmttkrp.so in-tree: host C++ with g++, kernels with hipcc for gfx950.

Run ``python -m paper_2405_08470_amd.build``.  Every call recompiles.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libspmttkrp.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
ARCH = "gfx950"

HOST_SOURCES = ["plan.cpp", "api.cpp"]
HIP_SOURCES = ["ec_n4.hip", "ec_n5.hip", "ec_n6.hip", "ec_n3.hip", "ec_n8.hip", "ec_n7.hip", "ec_n2.hip",
               "ec_kernel.hip", "dr_staged.hip", "als_kernels.hip", "grad_kernel.hip", "device_plan.hip",
               "probe.hip", "noalloc.hip"]

# Packed FP32 arithmetic is disabled for all device code: the compiler would
# otherwise emit v_pk_{add,mul,fma}_f32 from plain float code.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-mcode-object-version=5",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Werror=uninitialized", "-Werror=sometimes-uninitialized", "-Werror=return-type",
             "-I", INCLUDE, "-I", CSRC]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Winit-self", "-Werror=uninitialized",
              "-Werror=return-type", "-D__HIP_PLATFORM_AMD__",
              "-I", INCLUDE, "-I", CSRC, "-I", os.path.join(ROCM, "include")]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build step failed: {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False, out: str = LIB, defines=(), objdir: str = OBJ) -> str:
    """Compiles every source and links `out`; `defines` are extra -D flags."""
    os.makedirs(objdir, exist_ok=True)
    dflags = [f"-D{d}" for d in defines]
    jobs = []
    for s in HOST_SOURCES:
        o = os.path.join(objdir, s + ".o")
        jobs.append(["g++", *HOST_FLAGS, *dflags, "-c", os.path.join(CSRC, s), "-o", o])
    for s in HIP_SOURCES:
        o = os.path.join(objdir, s + ".o")
        jobs.append([HIPCC, *HIP_FLAGS, *dflags, "-c", os.path.join(CSRC, s), "-o", o])
    with ThreadPoolExecutor(max(1, min(8, len(jobs)))) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    objs = [os.path.join(objdir, s + ".o") for s in HOST_SOURCES + HIP_SOURCES]
    tmp = out + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
