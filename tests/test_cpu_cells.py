"""Pins for the algorithm-matched CPU cell-list baseline (CPU only): it must
compute the same forces as the brute-force FP64 oracle (it is only a faster
route to the same sum) and follow the oracle's integrator, so the benchmark's
GPU-to-CPU ratio compares equal work."""
import numpy as np
import pytest

import cpu_cells
import ljsynth


@pytest.fixture(scope="module")
def state():
    w = ljsynth.WORKLOADS["lj4k"]
    pos4, vel4, box = ljsynth.make_state(w, jitter_amp=0.05, shuffle=True)
    return w, pos4, vel4, box


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_forces_match_oracle(orc, state):
    w, pos4, vel4, box = state
    fo, _, _ = orc.forces(orc.params(box), pos4)
    _, _, f64 = cpu_cells.run(pos4, vel4, box, 0, precision="f64")
    _, _, f32 = cpu_cells.run(pos4, vel4, box, 0, precision="f32")
    assert _rel(f64, fo) < 1e-12
    assert _rel(f32.astype(np.float64), fo) < 1e-5


def test_steps_follow_oracle_integrator(orc, state):
    w, pos4, vel4, box = state
    po, vo, _ = orc.run(orc.params(box, dt=w.dt), pos4, vel4, 10)
    pc, vc, _ = cpu_cells.run(pos4, vel4, box, 10, precision="f64", dt=w.dt)
    d = pc - np.asarray(po)[:, :3]
    d -= box * np.round(d / box)
    assert np.abs(d).max() < 1e-9
    assert np.abs(vc - np.asarray(vo)[:, :3]).max() < 1e-8


def test_small_box_refused():
    pos = np.zeros((4, 3))
    with pytest.raises(ValueError):
        cpu_cells.run(pos, pos, 6.0, 1)  # 2 cells per dimension
