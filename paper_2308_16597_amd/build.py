"""Build the gfx950 HIP library libptlbm.so in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libptlbm.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("lattice.hip", "particles.hip", "copy.hip", "api.cpp", "serve.cpp")]


def hipcc_command(out=LIB, arch="gfx950"):
    return ["hipcc", f"--offload-arch={arch}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-ffp-contract=off", "-Wall", "-Wno-unused-function",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
            "-x", "hip", *SOURCES, "-o", out]


def build(verbose=False):
    cmd = hipcc_command()
    if verbose:
        print(" ".join(cmd), flush=True)
    tmp = LIB + ".tmp"
    cmd[-1] = tmp
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
