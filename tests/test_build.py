"""Build-level checks of the HIP code (CPU only: hipcc cross-compiles).

Every kernel must run without scratch (private) memory: a spilled or
dynamically indexed register array turns into per-lane global-memory traffic
in the inner loops. Packed FP32 instructions must not appear either.
"""
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0709_3225_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"


def _build_flags():
    """The library's own device flags (build.py loaded by path, without
    importing the package, which would load the library)."""
    import importlib.util

    spec = importlib.util.spec_from_file_location("_mdlj_build", os.path.join(ROOT, "paper_0709_3225_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return [f for f in mod.FLAGS if f not in ("-shared", "-fPIC", "-Wall")]


def _device_asm(src):
    cmd = [HIPCC, *_build_flags(), "-I", os.path.join(ROOT, "include"), "-I", CSRC, "--cuda-device-only", "-S",
           src, "-o", "-"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    return res.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
@pytest.mark.parametrize("src", sorted(glob.glob(os.path.join(CSRC, "*.hip"))), ids=os.path.basename)
def test_kernels_use_no_scratch_and_no_packed_fp32(src):
    asm = _device_asm(src)
    sizes = [int(v) for v in re.findall(r"\.private_segment_fixed_size:\s+(\d+)", asm)]
    assert all(v == 0 for v in sizes), f"scratch use in {os.path.basename(src)}: {sizes}"
    assert not re.search(r"\bv_pk_(add|mul|fma)_f32\b", asm)
    # the distance screen's matrix-core results stay in VGPRs (no copies out of AGPRs)
    assert "v_accvgpr_read" not in asm
