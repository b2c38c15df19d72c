"""GPU: md_forces_noalloc, the variant of md_build_cells + md_forces whose
workspace is the library's static device array (for callers that cannot
allocate), against the same two calls on a caller-owned workspace. Two calls
in a row, the second on a smaller system, so the second runs on an array that
still holds the first call's contents."""
import numpy as np
import pytest

import ljsynth

pytestmark = pytest.mark.gpu


def test_no_alloc_forces_equal_workspace_path():
    import torch

    from paper_0709_3225_amd import LJSystem
    from paper_0709_3225_amd import _lib as L

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    cases = [
        ("lj4k shuffled", ljsynth.make_state(ljsynth.WORKLOADS["lj4k"], jitter_amp=0.05, shuffle=True)[::2]),
        ("lj256 two cells", ljsynth.make_state(ljsynth.WORKLOADS["lj256_check"], jitter_amp=0.05)[::2]),
    ]
    for name, (pos4, box) in cases:
        n = len(pos4)
        print(f"[case] md_forces_noalloc {name} n={n} box={box}", flush=True)
        pos = torch.from_numpy(np.ascontiguousarray(pos4, dtype=np.float32)).cuda()
        s = LJSystem(n, box)
        s.load(pos, forces=False)
        ref = s.forces().cpu().numpy()
        assert s.check() == 0
        out = torch.full((n, 4), float("nan"), dtype=torch.float32, device="cuda")
        L.md_forces_noalloc(s.params, pos, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.isfinite(got).all()
        assert np.array_equal(got, ref)  # same kernels on the same layout: bitwise
