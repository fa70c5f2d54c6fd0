"""Compile the HIP library (csrc/) for gfx950 into paper_2103_03517_amd/libhmc.so.

hipcc cross-compiles without a GPU.  Packed FP32 instructions are disabled
for the device code, and multiply-adds are contracted only within a source
expression.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhmc.so")
CSRC = os.path.join(HERE, "csrc")
SOURCES = [os.path.join(CSRC, "hmc_api.cpp"), os.path.join(CSRC, "hmc_batch.cpp"),
           os.path.join(CSRC, "hmc_kernels.hip"), os.path.join(CSRC, "hmc_batch_kernels.hip"),
           os.path.join(CSRC, "hmc_masked_kernels.hip"), os.path.join(CSRC, "hmc_deep_kernels.hip"),
           os.path.join(CSRC, "hmc_static.hip")]
ARCH = os.environ.get("HMC_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def flags():
    # -ffp-contract=on: multiply-adds are fused only within one source
    # expression, so the same device function rounds identically in every
    # kernel it is inlined into (the single-lattice and the batch passes);
    # the default (fast) lets the backend fuse across statements depending on
    # the surrounding code.
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall", "-ffp-contract=on",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False) -> str:
    """Compiles every source to an object in parallel, then links."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    with tempfile.TemporaryDirectory(prefix="hmc_build_") as tmp:
        objs = [os.path.join(tmp, os.path.basename(src) + ".o") for src in SOURCES]
        cmds = [[hipcc()] + flags() + ["-c", src, "-o", obj] for src, obj in zip(SOURCES, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            results = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
        for c, r in zip(cmds, results):
            if r.stdout or r.stderr:
                print(r.stdout + r.stderr, end="", flush=True)
            if r.returncode != 0:
                raise subprocess.CalledProcessError(r.returncode, c)
        link = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
