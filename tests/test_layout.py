"""The population layout (csrc/lattice.h) on the host: with 8-byte values
the 14 arrays of a state lie in tiles of 64 nodes, array i at element
64 i + tix(k) of the state's block; otherwise array i is its own range.
Every (array, node) pair must own one element of its own inside the state,
for lattices from one row to 4032 x 4000 and the widest pitch.  Built with
the ROCm clang for the host alone (no GPU)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang not installed")
def test_every_array_and_node_owns_one_element(tmp_path):
    exe = str(tmp_path / "layout_check")
    src = os.path.join(ROOT, "tests", "layout_check.cpp")
    subprocess.run([CLANG, "-x", "hip", "--offload-host-only", "-std=c++17", "-O2",
                    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2308_16597_amd", "csrc"),
                    src, "-o", exe], check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "layout ok" in r.stdout
