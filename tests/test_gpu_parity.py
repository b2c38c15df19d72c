"""GPU parity: the HIP path through the C-ABI against the FP64 oracle.

Tolerances: forces within 1e-5 relative L2 (over all 3N components), energy
and virial within 1e-6 relative, neighbour sets identical. Every case names
itself on stdout before it touches the GPU.
"""
import json
import os

import numpy as np
import pytest

import ljsynth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

pytestmark = pytest.mark.gpu

FORCE_TOL = 1e-5
ENERGY_TOL = 1e-6


def _torch():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _system(n, box, **kw):
    from paper_0709_3225_amd import LJSystem

    return LJSystem(n, box, **kw)


def _dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_forces(pos4, box, vel4=None, **kw):
    s = _system(len(pos4), box, **kw)
    s.load(_dev(pos4), None if vel4 is None else _dev(vel4))
    f = s.forces().cpu().numpy()[:, :3].astype(np.float64)
    e = s.energy().cpu().numpy()
    assert s.check() == 0
    return s, f, e


def _clump_state():
    """Dense cubic block (spacing 0.53, 11^3 atoms) filling 2x2x2 cells of a
    12-sigma box: more than 64 atoms per home cell and a 27-cell
    neighbourhood larger than one LDS pass, next to empty cells. The spacing
    keeps every lattice distance at least 0.014 away from r_c."""
    g = np.arange(0.3, 5.9, 0.53)
    pts = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    rng = np.random.default_rng(9)
    pts = pts + rng.uniform(-0.002, 0.002, pts.shape)
    pos4 = np.zeros((len(pts), 4), np.float32)
    pos4[:, :3] = pts
    return pos4, 12.0


CASES = {
    "lj4k_jitter_shuffled": lambda: ljsynth.make_state(ljsynth.WORKLOADS["lj4k"], jitter_amp=0.05, shuffle=True)[::2],
    "lj256_two_cells": lambda: ljsynth.make_state(ljsynth.WORKLOADS["lj256_check"], jitter_amp=0.05)[::2],
    "lj32k_jitter": lambda: ljsynth.make_state(ljsynth.WORKLOADS["lj32k_adjoint"], jitter_amp=0.05)[::2],
    # 32 atoms in every cell: every round on the 32-column matrix layout
    "fcc_rho1.2_jitter": lambda: ljsynth.make_state(ljsynth.Workload("fcc_rho1.2", 10, 1.2, 1.0, 1, 7),
                                                    jitter_amp=0.05)[::2],
    "sparse_gas_rho0.05": lambda: _gas(1500, 0.05, 21),
    "fluid_rho0.4_ragged": lambda: _gas(2999, 0.4, 22, min_sep=0.8),
    "dense_clump": _clump_state,
}

# exactly k atoms in every cell of a 4^3 grid: the 12-slice VALU layout, three
# slices, two slices (compressed states with contacts near 0.72 sigma: pair
# sets and forces, not the energy bound)
LAYOUT_CASES = {
    "cells_of_5": lambda: ljsynth.k_per_cell(5, 305),
    "cells_of_18": lambda: ljsynth.k_per_cell(18, 318),
    "cells_of_22": lambda: ljsynth.k_per_cell(22, 322),
}


def _gas(n, rho, seed, min_sep=0.0):
    pos4, box = ljsynth.random_fluid(n, rho, seed)
    if min_sep > 0:  # drop atoms closer than min_sep to an earlier one (keeps forces moderate)
        keep = []
        pts = pos4[:, :3].astype(np.float64)
        for i in range(n):
            d = pts[keep] - pts[i] if keep else np.zeros((0, 3))
            d -= box * np.round(d / box)
            if not len(d) or (np.einsum("ij,ij->i", d, d) >= min_sep ** 2).all():
                keep.append(i)
        pos4 = pos4[keep]
    return pos4, box


@pytest.mark.parametrize("case", list(CASES))
def test_forces_and_energy_match_oracle(case, orc):
    pos4, box = CASES[case]()
    _say(f"forces {case} n={len(pos4)} box={box}")
    vel4 = np.zeros_like(pos4)
    vel4[:, :3] = np.random.default_rng(5).normal(size=(len(pos4), 3))
    _, f, e = gpu_forces(pos4, box, vel4)
    p = orc.params(box)
    fo, U, W = orc.forces(p, pos4)
    K = orc.kinetic(p, vel4)
    assert rel_l2(f, fo) <= FORCE_TOL
    assert abs(e[0] - U) <= ENERGY_TOL * abs(U)
    assert abs(e[1] - K) <= ENERGY_TOL * abs(K)
    assert abs(e[2] - W) <= ENERGY_TOL * abs(W)


@pytest.mark.parametrize("mode", [1])
def test_energy_shift_mode(mode, orc):
    pos4, vel4, box = ljsynth.make_state(ljsynth.WORKLOADS["lj4k"], jitter_amp=0.05)
    _say(f"shift_mode={mode} lj4k")
    _, f, e = gpu_forces(pos4, box, shift_mode=mode)
    fo, U, W = orc.forces(orc.params(box, shift_mode=mode), pos4)
    assert rel_l2(f, fo) <= FORCE_TOL
    assert abs(e[0] - U) <= ENERGY_TOL * abs(U)
    assert abs(e[2] - W) <= ENERGY_TOL * abs(W)


def test_energy_shift_mode_cutoff_sensitive_lj32k(orc):
    """With the plain truncated force (shift_mode 1) every pair dropped or
    added near r_c moves the force by |f_LJ(r_c)| = 0.039, far above the
    1e-5 gate: the whole N = 32,000 system (mostly cells of 11..16 atoms,
    screened on the matrix cores) against the oracle."""
    pos4, vel4, box = ljsynth.make_state(ljsynth.WORKLOADS["lj32k_adjoint"], jitter_amp=0.05)
    _say("shift_mode=1 lj32k whole system")
    _, f, e = gpu_forces(pos4, box, shift_mode=1)
    fo, U, W = orc.forces(orc.params(box, shift_mode=1), pos4)
    assert rel_l2(f, fo) <= FORCE_TOL
    assert abs(e[0] - U) <= ENERGY_TOL * abs(U)
    assert abs(e[2] - W) <= ENERGY_TOL * abs(W)


def test_energy_shift_mode_sampled_rows_lj256k(orc):
    """shift_mode 1 at N = 256,000: 2,048 sampled rows against the oracle's
    rows, each the full sum over all N atoms."""
    w = ljsynth.WORKLOADS["lj256k"]
    pos4, vel4, box = ljsynth.make_state(w, jitter_amp=0.05)
    _say("shift_mode=1 lj256k sampled rows")
    _, f, _ = gpu_forces(pos4, box, shift_mode=1)
    sel = np.random.default_rng(18).choice(w.n, size=2048, replace=False)
    fo, _, _ = orc.forces_rows(orc.params(box, shift_mode=1), pos4, sel)
    assert rel_l2(f[sel], fo) <= FORCE_TOL


NEIGHBOR_CASES = ["lj4k_jitter_shuffled", "lj256_two_cells", "lj32k_jitter", "fcc_rho1.2_jitter", "sparse_gas_rho0.05",
                  "fluid_rho0.4_ragged", "dense_clump"]


def _assert_rows(counts, idx, counts_o, idx_o):
    counts = counts.cpu().numpy()
    idx = idx.cpu().numpy()
    np.testing.assert_array_equal(counts, counts_o)
    off = np.concatenate([[0], np.cumsum(counts_o)])
    for i in range(len(counts_o)):
        assert np.array_equal(np.sort(idx[i, :counts[i]]), idx_o[off[i]:off[i + 1]]), i


@pytest.mark.parametrize("case", NEIGHBOR_CASES)
def test_neighbor_sets_exact(case, orc):
    """The pairs the force kernel's own walk accepts (its staging, matrix-core
    screen, bit walk and exact cutoff test; the export is a template variant
    of the force pass) equal the oracle's brute-force sets."""
    pos4, box = CASES[case]()
    _say(f"neighbors {case} n={len(pos4)}")
    counts_o, idx_o, guard = orc.neighbors(orc.params(box), pos4)
    assert guard == 0, "instance has pairs within the FP32/FP64 guard band of r_c"
    s = _system(len(pos4), box)
    s.load(_dev(pos4), forces=False)
    cap = int(counts_o.max()) + 8
    counts, idx = s.neighbors(cap)
    assert s.check() == 0
    _assert_rows(counts, idx, counts_o, idx_o)


@pytest.mark.parametrize("waves", [1, 4])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 16, 17, 20, 21, 22, 24])
def test_every_home_layout_matches_oracle(k, waves, orc):
    """Every cell holds exactly k atoms, so every home cell takes the same
    lane layout: the VALU screen with 16 down to 6 slices (k <= 10), the
    matrix-core screen (11..16), three and two slices (17..24; the larger
    neighbourhoods in more than one LDS pass). With the plain truncated force
    every pair dropped or added near r_c moves a force by |f_LJ(r_c)|; forces
    against the oracle, and the pairs the force kernel's walk accepts
    against its brute-force sets. One wavefront per cell, and four that
    split every pass's candidates between them."""
    pos4, box = ljsynth.k_per_cell(k, 100 + k)
    _say(f"home layout k={k} n={len(pos4)} waves={waves}")
    p = orc.params(box, shift_mode=1)
    counts_o, idx_o, guard = orc.neighbors(p, pos4)
    assert guard == 0, "instance has pairs within the FP32/FP64 guard band of r_c"
    s, f, _ = gpu_forces(pos4, box, shift_mode=1, waves_per_cell=waves)
    assert s.cells_per_dim == 4
    fo, _, _ = orc.forces(p, pos4)
    assert rel_l2(f, fo) <= FORCE_TOL
    counts, idx = s.neighbors(int(counts_o.max()) + 8)
    assert s.check() == 0
    _assert_rows(counts, idx, counts_o, idx_o)


@pytest.mark.parametrize("case", ["lj4k_jitter_shuffled", "lj32k_jitter", "fcc_rho1.2_jitter", "dense_clump",
                                  "cells_of_5", "cells_of_18", "cells_of_22"])
def test_neighbor_sets_pair_lists(case, orc):
    """The pair-list path of md_step_list: the pass that screens against the
    list radius and keeps the accept words, then the pass that walks the kept
    words, each export the oracle's sets (the dense clump takes several LDS
    passes and so screens in both)."""
    pos4, box = {**CASES, **LAYOUT_CASES}[case]()
    _say(f"neighbors via pair lists {case} n={len(pos4)}")
    counts_o, idx_o, guard = orc.neighbors(orc.params(box), pos4)
    assert guard == 0
    s = _system(len(pos4), box, pair_lists=True)
    s.load(_dev(pos4), forces=False)
    cap = int(counts_o.max()) + 8
    for mode in ("record", "kept"):
        counts, idx = s.neighbors(cap, lists=mode)
        assert s.check() == 0
        _assert_rows(counts, idx, counts_o, idx_o)


def _check_cell_lists(pos4, box, steps=0, vel4=None):
    s = _system(len(pos4), box)
    s.load(_dev(pos4), None if vel4 is None else _dev(vel4), forces=steps > 0)
    if steps:
        s.step(steps)
    start, order = s.cell_lists()
    pos, _ = s.state()
    assert s.check() == 0
    start = start.cpu().numpy()
    order = order.cpu().numpy()
    pos = pos.cpu().numpy()
    n, nc = len(pos4), s.cells_per_dim
    assert start[0] == 0 and start[-1] == n and np.all(np.diff(start) >= 0)
    assert np.array_equal(np.sort(order), np.arange(n))
    inv_s = np.float32(nc) / np.float32(box)
    ic = np.clip((pos[:, :3] * inv_s).astype(np.int64), 0, nc - 1)
    cell_of_atom = ic[:, 0] + nc * (ic[:, 1] + nc * ic[:, 2])
    cell_of_slot = np.repeat(np.arange(nc ** 3), np.diff(start))
    np.testing.assert_array_equal(cell_of_atom[order], cell_of_slot)
    # stable order inside each cell: ascending user index
    same = cell_of_slot[1:] == cell_of_slot[:-1]
    assert np.all(np.diff(order)[same] > 0)


@pytest.mark.parametrize("case", ["lj4k_jitter_shuffled", "sparse_gas_rho0.05", "dense_clump"])
def test_cell_lists_are_a_valid_counting_sort(case):
    pos4, box = CASES[case]()
    _say(f"cell lists {case} n={len(pos4)}")
    _check_cell_lists(pos4, box)


@pytest.mark.parametrize("name", ["lj256k", "lj2m"])
def test_cell_lists_full_size_after_steps(name):
    """Grids of 26^3 and 53^3 cells (one and several scan tiles), rebuilt by
    the fused drift of a 3-step run."""
    w = ljsynth.WORKLOADS[name]
    pos4, vel4, box = ljsynth.make_state(w, jitter_amp=0.05, shuffle=True)
    _say(f"cell lists full size {name} n={w.n}, 3 steps")
    _check_cell_lists(pos4, box, steps=3, vel4=vel4)


def _gas_with_cluster(box, n_gas, seed):
    """Ideal gas at low density plus a 10^3 simple-cubic cluster of spacing
    0.75 sigma in one corner: the cluster's cells hold about 40 atoms, past the
    bucket capacity of a dilute grid (32), so binning uses the overflow list.
    Gas atoms closer than 1 sigma to the cluster or to each other are dropped."""
    rng = np.random.default_rng(seed)
    g = 0.1 + 0.75 * np.arange(10)  # four planes inside the first cell on each axis
    cl = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pts = [p for p in cl]
    gas = rng.uniform(0, box, (n_gas, 3))
    for q in gas:
        d = np.asarray(pts) - q
        d -= box * np.round(d / box)
        if (np.einsum("ij,ij->i", d, d) >= 1.0).all():
            pts.append(q)
    pos4 = np.zeros((len(pts), 4), np.float32)
    pos4[:, :3] = np.asarray(pts)
    vel4 = np.zeros_like(pos4)
    vel4[:, :3] = rng.normal(0, 0.5, (len(pts), 3))
    return pos4, vel4, np.float32(box)


@pytest.mark.parametrize("box,n_gas", [(16.0, 100), (85.0, 3000)], ids=["direct_offsets", "block_scan"])
def test_bucket_overflow_build_and_steps(box, n_gas, orc):
    """Cells beyond the bucket capacity, on a grid whose cell order sums block
    counts itself (16 sigma, 6^3 cells) and on one that needs the block scan
    (85 sigma, 33^3 cells > 2048 blocks of 16): build, forces against the
    oracle, three fused steps, cell-list invariants and forces again."""
    pos4, vel4, box = _gas_with_cluster(box, n_gas, 31)
    _say(f"bucket overflow box={box} n={len(pos4)}")
    s = _system(len(pos4), box)
    s.load(_dev(pos4), _dev(vel4))
    f = s.forces().cpu().numpy()[:, :3]
    assert s.check() == 0
    fo, _, _ = orc.forces(orc.params(box), pos4)
    assert rel_l2(f, fo) <= FORCE_TOL
    s.step(3)
    pos, _ = s.state()
    f = s.forces().cpu().numpy()[:, :3]
    assert s.check() == 0
    p3 = pos.cpu().numpy()
    fo, _, _ = orc.forces(orc.params(box), p3)
    assert rel_l2(f, fo) <= FORCE_TOL
    _check_cell_lists(p3, box)


def _one_crowded_cell(seed=33):
    """4,096 atoms in one cell: a 16^3 simple-cubic block of spacing 15/16
    sigma, jittered by up to 0.09 sigma, filling the first of 27 cells of side
    16 sigma (box 48, cell_min 15.9), plus a dilute gas around it. The bucket
    capacity follows the mean occupancy (about 170 atoms per cell), so some
    3,900 atoms of that cell go through the overflow list on every build."""
    rng = np.random.default_rng(seed)
    g = 0.5 + (15.0 / 16.0) * np.arange(16)
    block = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    block = block + rng.uniform(-0.09, 0.09, block.shape)
    gas = rng.uniform(17.0, 47.0, (600, 3))
    keep = [q for i, q in enumerate(gas)
            if (np.einsum("ij,ij->i", gas[:i] - q, gas[:i] - q) >= 1.0).all()]
    pts = np.concatenate([block, np.asarray(keep)])
    pos4 = np.zeros((len(pts), 4), np.float32)
    pos4[:, :3] = pts
    vel4 = np.zeros_like(pos4)
    vel4[:, :3] = rng.normal(0.0, 0.3, (len(pts), 3))
    return pos4, vel4, np.float32(48.0)


def test_crowded_cell_builds_in_linear_time(orc):
    """A cell holding 4,096 atoms: its members past the bucket capacity are
    found through the per-cell overflow index, so a build, a force pass and
    three rebuilding steps finish in well under 5 s (the search of the whole
    overflow list for every member took minutes here); cell lists stay a
    valid counting sort and forces match the oracle."""
    import time

    torch = _torch()
    pos4, vel4, box = _one_crowded_cell()
    _say(f"crowded cell n={len(pos4)} box={box}")
    s = _system(len(pos4), box, cell_min=15.9, dt=1e-4)
    assert s.cells_per_dim == 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.load(_dev(pos4), _dev(vel4))
    s.step(3)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert s.check() == 0
    assert elapsed < 5.0, elapsed
    pos, _ = s.state()
    p3 = pos.cpu().numpy()
    f = s.forces().cpu().numpy()[:, :3]
    assert s.check() == 0
    fo, _, _ = orc.forces(orc.params(box), p3)
    assert rel_l2(f, fo) <= FORCE_TOL
    start, order = s.cell_lists()
    start = start.cpu().numpy()
    assert np.diff(start).max() == 4096
    assert np.array_equal(np.sort(order.cpu().numpy()), np.arange(len(pos4)))


@pytest.mark.parametrize("name", ["lj4k", "lj256k", "lj2m"])
def test_fcc_lattice_energy_pin(name):
    """Perfect FCC at rho = 0.8442: U/N = -5.693278, W/N = -20.16527 from the
    textbook shells (12, 6, 24, 12 sites inside r_c), with no oracle in the
    loop; every atom has the same environment, so the FP64 totals of the full
    systems must give these per-atom values to 1e-6."""
    w = ljsynth.WORKLOADS[name]
    pos4, vel4, box = ljsynth.make_state(w)
    _say(f"fcc lattice pin {name} n={w.n}")
    _, f, e = gpu_forces(pos4, box)
    assert e[0] / w.n == pytest.approx(-5.693278, rel=1e-6)
    assert e[2] / w.n == pytest.approx(-20.16527, rel=1e-6)
    assert np.abs(f).max() < 1e-3


def test_nve_run_and_parity_after_100_steps(orc):
    w = ljsynth.WORKLOADS["lj4k"]
    pos4, vel4, box = ljsynth.make_state(w)
    _say("nve lj4k 100 steps")
    s = _system(w.n, box, dt=w.dt)
    s.load(_dev(pos4), _dev(vel4))
    e0 = s.energy().cpu().numpy()
    th = s.step(100, thermo_every=1).cpu().numpy()
    assert s.check() == 0
    etot = np.concatenate([[e0[0] + e0[1]], th[:, 0] + th[:, 1]])
    assert np.abs(etot - etot[0]).max() / abs(etot[0]) < 5e-4
    # the oracle over the same 100 steps: energies agree closely early on
    _, _, tho = orc.run(orc.params(box, dt=w.dt), pos4, vel4, 100)
    eo = tho[:, 0] + tho[:, 1]
    assert abs(etot[10] - eo[10]) / abs(eo[10]) < 1e-5
    # feed the GPU state after 100 steps back to the oracle
    pos, vel = s.state()
    pos = pos.cpu().numpy()
    vel = vel.cpu().numpy()
    f = s.forces().cpu().numpy()[:, :3]
    e = s.energy().cpu().numpy()
    p = orc.params(box)
    fo, U, W = orc.forces(p, pos)
    assert rel_l2(f, fo) <= FORCE_TOL
    assert abs(e[0] - U) <= ENERGY_TOL * abs(U)
    assert abs(e[1] - orc.kinetic(p, vel)) <= ENERGY_TOL * abs(e[1])
    assert abs(e[2] - W) <= ENERGY_TOL * abs(W)
    np.testing.assert_allclose(th[-1], e, rtol=1e-12)


def test_long_nve_energy_conservation():
    """20,000 steps (100 tau) of the lj4k fluid from its FCC start: sampled
    every 100 steps, the total energy U + K stays within 1e-4 of its start
    and shows no secular drift (mean of the second half against the first
    within 2e-5). The paper prints no bound; it only notes that FP32 may not
    conserve energy. The FP32 rounding of the positions alone moves the energy
    by about sqrt(3N) |F| ulp(x) / sqrt(12) = 6.6e-4 per step in a random walk,
    0.07 (4e-6 relative) after 10^4 steps, so the halves may differ by a few
    1e-6 for any summation order without a systematic error; a missing or
    one-sided pair set drifts by orders of magnitude more. Measured on the
    MI355X: 2.4e-5 and 5e-7 with one force kernel, 5.1e-6 with another (the
    per-step excursion of the first steps from the lattice, up to 1.8e-4, is
    the 100-step test's)."""
    w = ljsynth.WORKLOADS["lj4k"]
    pos4, vel4, box = ljsynth.make_state(w)
    _say("nve lj4k 20000 steps")
    s = _system(w.n, box, dt=w.dt)
    s.load(_dev(pos4), _dev(vel4))
    e0 = s.energy().cpu().numpy()
    th = s.step(20000, thermo_every=100).cpu().numpy()
    assert s.check() == 0
    e_ref = e0[0] + e0[1]
    etot = th[:, 0] + th[:, 1]
    assert np.abs(etot - e_ref).max() / abs(e_ref) < 1e-4
    half = len(etot) // 2
    assert abs(etot[half:].mean() - etot[:half].mean()) / abs(e_ref) < 2e-5


def test_single_step_matches_oracle_step(orc):
    w = ljsynth.WORKLOADS["lj4k"]
    pos4, vel4, box = ljsynth.make_state(w, jitter_amp=0.05)
    _say("one step lj4k")
    s = _system(w.n, box, dt=w.dt)
    s.load(_dev(pos4), _dev(vel4))
    s.step(1)
    pos, vel = s.state()
    assert s.check() == 0
    x, v, _ = orc.run(orc.params(box, dt=w.dt), pos4, vel4, 1)
    d = pos.cpu().numpy()[:, :3] - x
    d -= box * np.round(d / box)
    assert np.abs(d).max() < 2e-5
    assert rel_l2(vel.cpu().numpy()[:, :3], v) < 1e-5


def test_bitwise_deterministic():
    w = ljsynth.WORKLOADS["lj4k"]
    pos4, vel4, box = ljsynth.make_state(w, shuffle=True)
    _say("determinism lj4k 20 steps x2")
    outs = []
    for _ in range(2):
        s = _system(w.n, box)
        s.load(_dev(pos4), _dev(vel4))
        s.step(20)
        pos, vel = s.state()
        f = s.forces()
        e = s.energy()
        assert s.check() == 0
        outs.append([t.cpu().numpy() for t in (pos, vel, f, e)])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_step_chunks_equal_one_call():
    """Inside one md_step call every force pass but the last also performs the
    next step's half kick and drift; a call of one step runs the separate drift
    kernel. Any split of the same run must give bitwise the same state."""
    w = ljsynth.WORKLOADS["lj4k"]
    pos4, vel4, box = ljsynth.make_state(w, jitter_amp=0.05, shuffle=True)
    _say("step chunks lj4k")
    res = []
    for chunks in ([10], [3, 7], [1] * 10):
        s = _system(w.n, box)
        s.load(_dev(pos4), _dev(vel4))
        for c in chunks:
            s.step(c)
        pos, vel = s.state()
        res.append([t.cpu().numpy() for t in (pos, vel, s.forces(), s.energy())])
        assert s.check() == 0
    for other in res[1:]:
        for a, b in zip(res[0], other):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("name,rows", [("lj256k", 1024), ("lj2m", 512)])
def test_full_size_sampled_rows(name, rows, orc):
    w = ljsynth.WORKLOADS[name]
    pos4, vel4, box = ljsynth.make_state(w, jitter_amp=0.05)
    _say(f"full size {name} n={w.n} rows={rows}")
    _, f, e = gpu_forces(pos4, box, vel4)
    sel = np.random.default_rng(17).choice(w.n, size=rows, replace=False)
    fo, ur, wr = orc.forces_rows(orc.params(box), pos4, sel)
    assert rel_l2(f[sel], fo) <= FORCE_TOL
    if name == "lj256k":
        # the full O(N^2) oracle sums of this state, stored once by
        # tests/golden/make_full_energy.py (the FCC pin covers N = 2,048,000)
        g = json.load(open(os.path.join(GOLDEN, "lj256k_jitter_energy.json")))
        assert g["n"] == w.n and g["jitter"] == 0.05 and g["box"] == box
        assert abs(e[0] - g["U"]) <= ENERGY_TOL * abs(g["U"])
        assert abs(e[2] - g["W"]) <= ENERGY_TOL * abs(g["W"])


WAVE_CASES = ["lj4k_jitter_shuffled", "lj256_two_cells", "lj32k_jitter", "fcc_rho1.2_jitter", "sparse_gas_rho0.05",
              "fluid_rho0.4_ragged", "dense_clump"]


@pytest.mark.parametrize("waves", [2, 4])
@pytest.mark.parametrize("case", WAVE_CASES)
def test_waves_per_cell_match_oracle(case, waves, orc):
    """Two or four wavefronts per home cell split each pass's candidates
    (matrix-core blocks or VALU groups, at multiples of the screen's step) and
    add their partials in wavefront order: forces and energies against the
    oracle at the same bar as one wavefront; the cases span the matrix-core
    and VALU screens, face and interior cells, several passes (dense_clump)
    and ranges that leave a wavefront no candidates (sparse gas)."""
    pos4, box = CASES[case]()
    _say(f"waves {waves} {case} n={len(pos4)}")
    vel4 = np.zeros_like(pos4)
    vel4[:, :3] = np.random.default_rng(5).normal(size=(len(pos4), 3))
    _, f, e = gpu_forces(pos4, box, vel4, waves_per_cell=waves)
    _, f1, e1 = gpu_forces(pos4, box, vel4, waves_per_cell=1)
    p = orc.params(box)
    fo, U, W = orc.forces(p, pos4)
    K = orc.kinetic(p, vel4)
    assert rel_l2(f, fo) <= FORCE_TOL
    assert abs(e[0] - U) <= ENERGY_TOL * abs(U)
    assert abs(e[1] - K) <= ENERGY_TOL * abs(K)
    assert abs(e[2] - W) <= ENERGY_TOL * abs(W)
    # the same pairs as one wavefront: only the order of the FP32 sums differs
    assert rel_l2(f, f1) <= 1e-6
    assert e[1] == e1[1]


@pytest.mark.parametrize("tile", [128, 192, 1024])
@pytest.mark.parametrize("case", ["lj4k_jitter_shuffled", "lj32k_jitter", "dense_clump", "fluid_rho0.4_ragged"])
def test_tile_cap_matches_oracle(case, tile, orc):
    """The LDS tile knob: a tile of 128 or 192 atoms splits every 27-cell
    neighbourhood of the dense states into several passes (the cursor
    staging of every cell, interior ones included), a 1,024-atom tile keeps
    the clump's in one; forces and energies against the oracle at the usual
    bar, and the same pairs as the formula's tile (only the order of the FP32
    sums differs), in one and in four wavefronts per cell."""
    from paper_0709_3225_amd import _lib as L

    pos4, box = CASES[case]()
    _say(f"tile {tile} {case} n={len(pos4)}")
    vel4 = np.zeros_like(pos4)
    vel4[:, :3] = np.random.default_rng(6).normal(size=(len(pos4), 3))
    p = orc.params(box)
    fo, U, W = orc.forces(p, pos4)
    K = orc.kinetic(p, vel4)
    _, f0, e0 = gpu_forces(pos4, box, vel4)
    for waves in (1, 4):
        s, f, e = gpu_forces(pos4, box, vel4, tile_cap=tile, waves_per_cell=waves)
        assert L.md_tile_capacity(s.params) == tile
        assert rel_l2(f, fo) <= FORCE_TOL
        assert abs(e[0] - U) <= ENERGY_TOL * abs(U)
        assert abs(e[1] - K) <= ENERGY_TOL * abs(K)
        assert abs(e[2] - W) <= ENERGY_TOL * abs(W)
        assert rel_l2(f, f0) <= 1e-6
        assert e[1] == e0[1]


def test_tile_cap_steps_repeatable(orc):
    """md_step with a 192-atom tile: one step against the oracle's step and
    two 20-step runs bitwise equal."""
    torch = _torch()
    w = ljsynth.WORKLOADS["lj4k"]
    pos4, vel4, box = ljsynth.make_state(w, jitter_amp=0.05, shuffle=True)
    _say("tile 192 steps lj4k")
    runs = []
    for _ in range(2):
        s = _system(w.n, box, dt=w.dt, tile_cap=192)
        s.load(_dev(pos4), _dev(vel4))
        s.step(1)
        if not runs:
            pos, vel = s.state()
            x, v, _ = orc.run(orc.params(box, dt=w.dt), pos4, vel4, 1)
            d = pos.cpu().numpy()[:, :3] - x
            d -= box * np.round(d / box)
            assert np.abs(d).max() < 2e-5
            assert rel_l2(vel.cpu().numpy()[:, :3], v) < 1e-5
        s.step(19)
        assert s.check() == 0
        runs.append(s.state())
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][1], runs[1][1])


@pytest.mark.parametrize("waves", [2, 4])
def test_waves_per_cell_steps(waves, orc):
    """md_step with several wavefronts per cell: one step against the oracle's
    step, a 20-step run bitwise repeatable, and the no-rebuild and batched
    paths (which share the force pass) on the same state."""
    w = ljsynth.WORKLOADS["lj4k"]
    pos4, vel4, box = ljsynth.make_state(w, jitter_amp=0.05, shuffle=True)
    _say(f"waves {waves} steps lj4k")
    s = _system(w.n, box, dt=w.dt, waves_per_cell=waves)
    s.load(_dev(pos4), _dev(vel4))
    s.step(1)
    pos, vel = s.state()
    assert s.check() == 0
    x, v, _ = orc.run(orc.params(box, dt=w.dt), pos4, vel4, 1)
    d = pos.cpu().numpy()[:, :3] - x
    d -= box * np.round(d / box)
    assert np.abs(d).max() < 2e-5
    assert rel_l2(vel.cpu().numpy()[:, :3], v) < 1e-5
    outs = []
    for _ in range(2):
        s = _system(w.n, box, dt=w.dt, waves_per_cell=waves)
        s.load(_dev(pos4), _dev(vel4))
        th = s.step(20, thermo_every=10)
        pos, vel = s.state()
        assert s.check() == 0
        outs.append([t.cpu().numpy() for t in (pos, vel, th)])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
    # the 20-step energies of one wavefront, to FP32 round-off of the trajectory
    s1 = _system(w.n, box, dt=w.dt, waves_per_cell=1)
    s1.load(_dev(pos4), _dev(vel4))
    th1 = s1.step(20, thermo_every=10).cpu().numpy()
    e_w = outs[0][2][:, 0] + outs[0][2][:, 1]
    e_1 = th1[:, 0] + th1[:, 1]
    assert np.abs(e_w - e_1).max() / abs(e_1[0]) < 1e-5
    # steps between rebuilds (md_step_every, skin 0.86) take the same force pass
    se = _system(w.n, box, dt=w.dt, cell_min=2.9, waves_per_cell=waves)
    se.load(_dev(pos4), _dev(vel4))
    te = se.step_every(20, 5, thermo_every=10).cpu().numpy()
    assert se.check() == 0
    _, _, tho = orc.run(orc.params(box, dt=w.dt), pos4, vel4, 20)
    eo = tho[:, 0] + tho[:, 1]
    assert np.abs(te[:, 0] + te[:, 1] - eo[[10, 20]]).max() / abs(eo[0]) < 1e-5


def test_waves_per_cell_batched(orc):
    """A batch of replicas with four wavefronts per cell: each replica's
    forces against the oracle."""
    from paper_0709_3225_amd.batch import BatchedLJ

    torch = _torch()
    w = ljsynth.WORKLOADS["lj4k"]
    states = [ljsynth.make_state(w, jitter_amp=0.05), ljsynth.make_state(ljsynth.WORKLOADS["lj256_check"],
                                                                        jitter_amp=0.05)]
    _say("waves 4 batched lj4k + lj256")
    b = BatchedLJ([(len(p), box) for p, _, box in states], waves_per_cell=4)
    pos = torch.cat([_dev(p) for p, _, _ in states])
    vel = torch.cat([_dev(v) for _, v, _ in states])
    b.load(pos, vel)
    out = torch.empty((len(pos), 4), dtype=torch.float32, device="cuda")
    f = b.forces(out).cpu().numpy()[:, :3].astype(np.float64)
    b.check()
    off = 0
    for p4, _, box in states:
        fo, _, _ = orc.forces(orc.params(box), p4)
        assert rel_l2(f[off:off + len(p4)], fo) <= FORCE_TOL
        off += len(p4)


@pytest.mark.parametrize("case", ["lj4k_jitter_shuffled", "lj32k_jitter", "fluid_rho0.4_ragged"])
def test_thermo_temperature_and_pressure(case, orc):
    """md_thermo: U, K, W bitwise those of md_energy_virial, and T =
    2K / (3N - 3), P = (2K + W) / (3V) against the oracle's K and W."""
    pos4, box = CASES[case]()
    n = len(pos4)
    _say(f"thermo {case} n={n}")
    vel4 = np.zeros_like(pos4)
    vel4[:, :3] = np.random.default_rng(8).normal(scale=0.8, size=(n, 3))
    s = _system(n, box)
    s.load(_dev(pos4), _dev(vel4))
    t5 = s.thermo().cpu().numpy()
    e3 = s.energy().cpu().numpy()
    assert s.check() == 0
    assert np.array_equal(t5[:3], e3)
    p = orc.params(box)
    _, U, W = orc.forces(p, pos4)
    K = orc.kinetic(p, vel4)
    V = float(np.float32(box)) ** 3
    assert abs(t5[3] - 2.0 * K / (3 * n - 3)) <= ENERGY_TOL * (2.0 * K / (3 * n - 3))
    pref = (2.0 * K + W) / (3.0 * V)
    assert abs(t5[4] - pref) <= ENERGY_TOL * (2.0 * K + abs(W)) / (3.0 * V)


def test_edge_small_systems(orc):
    _say("edge: one atom, two atoms across the boundary")
    s, f, e = gpu_forces(np.array([[1.0, 2.0, 3.0, 0.0]], np.float32), 6.0)
    assert np.all(f == 0) and e[0] == 0 and e[2] == 0
    pos4 = np.array([[0.2, 5.0, 5.0, 0.0], [9.3, 5.0, 5.0, 0.0]], np.float32)
    _, f, e = gpu_forces(pos4, 10.0)
    fo, U, W = orc.forces(orc.params(10.0), pos4)
    assert rel_l2(f, fo) <= FORCE_TOL
    assert f[0, 0] > 0


def test_device_error_bits():
    torch = _torch()
    from paper_0709_3225_amd import _lib

    _say("error bits: step before forces, non-finite input")
    w = ljsynth.WORKLOADS["lj256_check"]
    pos4, vel4, box = ljsynth.make_state(w)
    s = _system(w.n, box)
    s.load(_dev(pos4), forces=False)
    s.step(2)
    assert s.check(raise_on_error=False) == _lib.MD_DEV_ORDER
    assert s.check() == 0  # cleared
    s.forces()
    s.step(2)
    assert s.check() == 0
    bad = pos4.copy()
    bad[3, 1] = np.nan
    s.load(_dev(bad), forces=False)
    assert s.check(raise_on_error=False) & _lib.MD_DEV_NONFINITE
    pos, _ = s.state()
    assert torch.isfinite(pos).all()
