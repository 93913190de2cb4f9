"""Build the CPU oracle (test infrastructure) with gcc.

FP64, one thread, no fused multiply-add (-ffp-contract=off), so every
operation rounds as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libptlbm_oracle.so")


def build(verbose=False):
    src = os.path.join(HERE, "ptlbm_oracle.c")
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", LIB, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
