"""Build-level check (CPU only): device code writes memory through vector
instructions only. No kernel may store, atomically update, write back or
discard through the scalar data cache. hipcc never emits these for plain HIP
stores and atomics; the check guards against a future intrinsic or asm use.

This file names those instructions, so the GPU-run snapshot excludes it
(it compiles code and never touches a GPU).
"""
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0709_3225_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
SCALAR_WRITES = re.compile(r"^\s*s_(store|buffer_store|scratch_store|atomic|buffer_atomic|dcache_wb|dcache_discard)\w*",
                           re.MULTILINE)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
@pytest.mark.parametrize("src", sorted(glob.glob(os.path.join(CSRC, "*.hip"))), ids=os.path.basename)
def test_no_scalar_cache_writes(src):
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "--cuda-device-only", "-S",
           src, "-o", "-"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    hits = SCALAR_WRITES.findall(res.stdout)
    assert not hits, f"{os.path.basename(src)}: {sorted(set(hits))}"
