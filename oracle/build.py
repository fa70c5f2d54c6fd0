"""Compile the CPU reference (test infrastructure) into oracle/liboracle.so.

Plain C11, gcc -O2, no fast-math and no FMA contraction, so every
operation rounds as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "hmc_oracle.c")]


SAN_LIB = os.path.join(HERE, "liboracle_san.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """sanitize: an AddressSanitizer + UndefinedBehaviorSanitizer build into
    liboracle_san.so (loaded by oracle.py when ORACLE_LIB names it, with the
    ASan runtime preloaded into the Python process)."""
    out = SAN_LIB if sanitize else LIB
    san = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"]
    cmd = ["gcc", "-std=c11"] + san + ["-fPIC", "-shared", "-ffp-contract=off",
                                        "-Wall", "-Wextra", "-o", out + ".tmp"] + SOURCES + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv)
    sys.exit(0)
