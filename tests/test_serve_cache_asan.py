"""The batch bookkeeping of lbm_step_many and lbm_step_many_noalloc
(csrc/serve.cpp), compiled for the host alone with AddressSanitizer against
the stub HIP runtime of serve_harness.cpp, which checks every event,
stream, graph, allocation and launched run table it is handed.  Runs are
created, stepped in random subsets (the caller's stream or a run's own),
re-seeded and destroyed in a seeded random order; the cache's graph
replays and LRU evictions happen along the way.  Nothing is used after it
is freed, every launched block names a live run, and everything the cache
held is released once its runs are destroyed."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"


def _build(out):
    inc = os.path.join(ROOT, "include")
    csrc = os.path.join(ROOT, "paper_2308_16597_amd", "csrc")
    flags = ["-x", "hip", "--offload-host-only", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address", "-I", inc, "-I", csrc, "-c"]
    objs = []
    for src in (os.path.join(csrc, "serve.cpp"), os.path.join(ROOT, "tests", "serve_harness.cpp")):
        o = os.path.join(out, os.path.basename(src) + ".o")
        subprocess.run([CLANG, *flags, src, "-o", o], check=True, capture_output=True)
        objs.append(o)
    # the host object names the (absent) device image; point it at a placeholder
    syms = subprocess.run(["nm", objs[0]], check=True, capture_output=True, text=True).stdout
    extra = [f"-Wl,--defsym={m}=harness_fatbin_placeholder" for m in re.findall(r" U (__hip_fatbin\w*)", syms)]
    exe = os.path.join(out, "harness")
    subprocess.run([CLANG, "-fsanitize=address", "-o", exe, *objs, *extra], check=True, capture_output=True)
    return exe


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang not installed")
def test_batch_cache_under_asan(tmp_path):
    exe = _build(str(tmp_path))
    for seed in (1, 2, 3):
        r = subprocess.run([exe, str(seed), "3000"], capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-4000:]
        assert "harness ok" in r.stdout, r.stdout
        # everything a batch held is released once its runs are gone (the two
        # events of the fixed-array path stay, by design, until the process ends)
        assert "2 events, 0 graphs, 0 executables, 0 allocations left" in r.stdout, r.stdout
        m = re.search(r"(\d+) cached and (\d+) fixed-array calls, (\d+) launches", r.stdout)
        assert m and int(m.group(1)) > 500 and int(m.group(2)) > 200 and int(m.group(3)) > 10000
