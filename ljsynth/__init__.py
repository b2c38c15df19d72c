"""Seeded synthetic inputs for Lennard-Jones fluids.

This module is shared by the tests, the benchmark and the smoke check. It
holds only input generation: lattice placement, random velocities, jitter and
the table of workload shapes. It computes no pair force, energy, cell list or
integration step; those live in the product library and, independently, in
the reference oracle.

Reduced LJ units throughout (epsilon = sigma = m = 1 unless a config says
otherwise). The paper measures synthetic LJ systems at densities up to 1.0 with
cutoff 2.5 sigma (section 3.2); the workloads below follow those shapes.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Workload",
    "WORKLOADS",
    "box_length",
    "fcc_positions",
    "maxwell_boltzmann",
    "jitter",
    "wrap_fp32",
    "make_state",
    "batched_replicas",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic LJ workload: an FCC crystal of n_fcc^3 unit cells."""

    name: str
    n_fcc: int
    density: float
    temperature: float
    steps: int
    seed: int
    dt: float = 0.005
    epsilon: float = 1.0
    sigma: float = 1.0
    mass: float = 1.0
    rc_over_sigma: float = 2.5
    shift_mode: int = 0  # 0: force shifted to zero at r_c; 1: energy shifted (WCA)

    @property
    def n(self) -> int:
        return 4 * self.n_fcc ** 3


# The workloads: parity case, single-GPU headline case, full-size case and the
# adjoint case with its small check instance.
WORKLOADS = {
    "lj4k": Workload("lj4k", 10, 0.8442, 1.0, 100, 1),
    "lj256k": Workload("lj256k", 40, 0.8442, 0.722, 1000, 2),
    "lj2m": Workload("lj2m", 80, 0.8442, 1.0, 500, 3),
    "lj32k_adjoint": Workload("lj32k_adjoint", 20, 0.8442, 1.0, 200, 5),
    "lj256_check": Workload("lj256_check", 4, 0.8442, 1.0, 200, 5),
}


# Widened workloads. The density axis of the paper's cell-list measurements
# (section 3.2, rho from 0.1 to 1.0) at the headline size, and WCA: LJ cut at
# its minimum 2^(1/6) sigma and shifted by eps (a short-range pair potential
# in place of LJ, as the paper's closing section allows). The WCA cutoff is
# the FP32 value both the GPU path and the oracle use.
DENSITY_SWEEP = (0.1, 0.2, 0.4, 0.6, 0.8442, 1.0)
WCA_RC = float(np.float32(2.0 ** (1.0 / 6.0)))


def sweep_workload(density: float, n_fcc: int = 40, seed: int = 40) -> Workload:
    return Workload(f"lj{4 * n_fcc ** 3 // 1000}k_rho{density}", n_fcc, density, 0.722, 100, seed)


def wca_workload(n_fcc: int = 40, density: float = 0.8442, seed: int = 41) -> Workload:
    return Workload(f"wca{4 * n_fcc ** 3 // 1000}k_rho{density}", n_fcc, density, 0.722, 100, seed,
                    rc_over_sigma=WCA_RC, shift_mode=1)


def box_length(n: int, density: float) -> float:
    """Cubic box side L = (N/rho)^(1/3), rounded once to FP32.

    Both the GPU path and the oracle take this FP32 value (widened to double
    on the CPU side) so that periodic images agree exactly.
    """
    return float(np.float32((n / density) ** (1.0 / 3.0)))


def wrap_fp32(x: np.ndarray, box: float) -> np.ndarray:
    """Bring FP32 coordinates into [0, L) after input perturbation."""
    L = np.float32(box)
    x = np.asarray(x, dtype=np.float32)
    x = (x - L * np.floor(x / L)).astype(np.float32)
    x = np.where(x >= L, x - L, x).astype(np.float32)
    x = np.where((x < 0) | (x >= L), np.float32(0), x).astype(np.float32)
    return x


def fcc_positions(n_fcc: int, box: float) -> np.ndarray:
    """FCC lattice of n_fcc^3 cubic unit cells filling the box.

    Four-atom basis {(0,0,0), (1/2,1/2,0), (1/2,0,1/2), (0,1/2,1/2)} times the
    lattice constant a = L/n_fcc, offset by a/4 on every axis so that no
    lattice plane lies on a cell boundary. Returns float64 [N, 3] in [0, L).
    """
    a = box / n_fcc
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    g = np.arange(n_fcc, dtype=np.float64)
    cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    pos = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a + 0.25 * a
    return pos


def maxwell_boltzmann(n: int, temperature: float, mass: float, seed: int) -> np.ndarray:
    """Gaussian velocities N(0, T/m) per component, zero net momentum,
    rescaled so that 2K/(3N-3) equals T exactly. Float64 [N, 3]."""
    rng = np.random.default_rng(seed)
    v = rng.normal(0.0, math.sqrt(temperature / mass), size=(n, 3))
    if n > 1:
        v -= v.mean(axis=0)
        k2 = (v * v).sum()  # twice the kinetic energy divided by the mass
        if k2 > 0:
            v *= math.sqrt(temperature * (3 * n - 3) / (mass * k2))
    else:
        v[:] = 0.0
    return v


def jitter(pos: np.ndarray, amplitude: float, seed: int) -> np.ndarray:
    """Uniform displacement in [-amplitude, amplitude) per coordinate."""
    rng = np.random.default_rng(seed)
    return pos + rng.uniform(-amplitude, amplitude, size=pos.shape)


def make_state(w: Workload, jitter_amp: float = 0.0, shuffle: bool = False):
    """Build (pos4, vel4, box) as FP32 numpy arrays of shape [N, 4].

    The w component is zero. ``jitter_amp`` > 0 adds the parity-only jitter
    (seeded with seed + 1000); ``shuffle`` applies a seeded permutation of the
    atom order (seed + 2000) so that user order is unrelated to space.
    """
    box = box_length(w.n, w.density)
    pos = fcc_positions(w.n_fcc, box)
    if jitter_amp > 0:
        pos = jitter(pos, jitter_amp, w.seed + 1000)
    vel = maxwell_boltzmann(w.n, w.temperature, w.mass, w.seed)
    if shuffle:
        perm = np.random.default_rng(w.seed + 2000).permutation(w.n)
        pos, vel = pos[perm], vel[perm]
    pos4 = np.zeros((w.n, 4), dtype=np.float32)
    vel4 = np.zeros((w.n, 4), dtype=np.float32)
    pos4[:, :3] = wrap_fp32(pos.astype(np.float32), box)
    vel4[:, :3] = vel.astype(np.float32)
    return pos4, vel4, box


def random_fluid(n: int, density: float, seed: int):
    """Uniformly random positions in the box (an ideal-gas snapshot).

    Used for edge cases: sparse and ragged cell occupancy, empty cells. Pairs
    can sit very close, so only small forces-parity cases use it with a
    minimum-separation filter applied by the caller if needed.
    """
    box = box_length(n, density)
    rng = np.random.default_rng(seed)
    pos4 = np.zeros((n, 4), dtype=np.float32)
    pos4[:, :3] = wrap_fp32(rng.uniform(0.0, box, size=(n, 3)).astype(np.float32), box)
    return pos4, box


def k_per_cell(k: int, seed: int, nc: int = 4, side: float = 2.6, rc: float = 2.5):
    """Exactly k <= 27 atoms in every cell of an nc^3 grid of side `side`
    (>= rc): each cell's atoms on k of the 27 sites of a 3^3 sub-lattice
    (spacing 0.35 side, 0.3 side across cell faces), picked at random per
    cell, with a uniform jitter of +-0.03, drawn again (next seed) while any
    pair lies within 2e-5 of rc. Returns (pos4, box). Every home cell then
    holds the same number of atoms, which fixes the kernels' lane layout."""
    box = nc * side
    u = np.array([0.15, 0.5, 0.85]) * side
    sites = np.stack(np.meshgrid(u, u, u, indexing="ij"), -1).reshape(-1, 3)
    cells = np.stack(np.meshgrid(*(np.arange(nc),) * 3, indexing="ij"), -1).reshape(-1, 3) * side
    for attempt in range(100):
        rng = np.random.default_rng(seed + 1000 * attempt)
        pts = np.concatenate([c + sites[rng.choice(27, size=k, replace=False)] for c in cells])
        pts += rng.uniform(-0.03, 0.03, pts.shape)
        pos4 = np.zeros((len(pts), 4), np.float32)
        pos4[:, :3] = pts
        d = pos4[:, None, :3].astype(np.float64) - pos4[None, :, :3].astype(np.float64)
        d -= box * np.round(d / box)
        r = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
        if not (np.abs(r - rc) < 2e-5).any():
            return pos4, box
    raise ValueError("no instance clear of rc")


def batched_replicas(count: int = 512, seed: int = 4):
    """Replica table of the batched workload: N = 4 n^3 with n uniform in
    [5, 20], density uniform in [0.70, 0.95], T uniform in [0.7, 1.5]."""
    rng = np.random.default_rng(seed)
    n_fcc = rng.integers(5, 21, size=count)
    rho = rng.uniform(0.70, 0.95, size=count)
    temp = rng.uniform(0.7, 1.5, size=count)
    return [
        Workload(f"replica{i}", int(n_fcc[i]), float(rho[i]), float(temp[i]), 200, seed * 100000 + i)
        for i in range(count)
    ]
