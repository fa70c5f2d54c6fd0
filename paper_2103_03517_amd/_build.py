"""Compile the HIP library (csrc/) for gfx950 into paper_2103_03517_amd/libhmc.so.

hipcc cross-compiles without a GPU.  Packed FP32 instructions are disabled
for the device code.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhmc.so")
CSRC = os.path.join(HERE, "csrc")
SOURCES = [os.path.join(CSRC, "hmc_api.cpp"), os.path.join(CSRC, "hmc_batch.cpp"),
           os.path.join(CSRC, "hmc_kernels.hip")]
ARCH = os.environ.get("HMC_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False) -> str:
    cmd = [hipcc()] + flags() + ["-shared", "-o", LIB + ".tmp"] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
