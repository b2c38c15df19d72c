"""A thin Python owner of one LJ system on the GPU.

Holds the parameters and the workspace tensor and forwards to the C-ABI
entry points; it computes nothing itself.
"""
from __future__ import annotations

import torch

from . import _lib as L


def occupancy_cell_min(n: int, box: float, rc: float, target: float = 14.0) -> float:
    """Cell side holding about ``target`` atoms on average at this density,
    never below r_c (section 3 asks only for cells of side >= r_c). With cells
    of side r_c at low density or with a short cutoff, a cell holds one or two
    atoms and a wavefront per home cell leaves most of its lanes idle; the
    value goes to ``cell_min``."""
    return max(float(rc), (float(target) * float(box) ** 3 / float(n)) ** (1.0 / 3.0))


class LJSystem:
    """Cubic periodic LJ system of n particles in a box of side ``box``."""

    def __init__(self, n, box, *, epsilon=1.0, sigma=1.0, mass=1.0, rc_over_sigma=2.5, dt=0.005,
                 cell_min=0.0, shift_mode=0, pair_lists=False, atom_lists=False, waves_per_cell=0, list_radius=0.0,
                 tile_cap=0, device="cuda"):
        flags = (L.MD_FLAG_PAIR_LISTS if pair_lists else 0) | (L.MD_FLAG_ATOM_LISTS if atom_lists else 0)
        self.params = L.make_params(n, box, epsilon, sigma, mass, rc_over_sigma, dt, cell_min, shift_mode, flags,
                                    waves_per_cell, list_radius, tile_cap)
        self.cells_per_dim, self.cell_side = L.md_cell_grid(self.params)  # raises on invalid params
        self.nbytes = L.md_workspace_bytes(self.params)
        self.device = torch.device(device)
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        self.n = int(n)

    @property
    def n_cells(self) -> int:
        return self.cells_per_dim ** 3

    def load(self, pos4: torch.Tensor, vel4: torch.Tensor | None = None, forces: bool = True):
        """md_build_cells on the given state, then (by default) md_forces."""
        L.md_build_cells(self.params, self.ws, pos4.contiguous(), None if vel4 is None else vel4.contiguous())
        if forces:
            L.md_forces(self.params, self.ws)

    def forces(self, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty((self.n, 4), dtype=torch.float32, device=self.device)
        L.md_forces(self.params, self.ws, out)
        return out

    def step(self, nsteps: int, thermo_every: int = 0, thermo_out: torch.Tensor | None = None):
        """md_step; with thermo_every > 0, (U, K, W) of every thermo_every-th
        step in FP64, into thermo_out if given (at least nsteps //
        thermo_every rows of 3 doubles) or a new tensor."""
        thermo = None
        if thermo_every > 0 and nsteps >= thermo_every:
            thermo = thermo_out
            if thermo is None:
                thermo = torch.empty((nsteps // thermo_every, 3), dtype=torch.float64, device=self.device)
        L.md_step(self.params, self.ws, nsteps, thermo_every if thermo is not None else 0, thermo)
        return thermo

    def step_every(self, nsteps: int, rebuild_every: int, thermo_every: int = 0):
        """md_step_every: cell lists rebuilt every rebuild_every steps (the
        skin is cell_side - r_c; choose it with cell_min)."""
        thermo = None
        if thermo_every > 0 and nsteps >= thermo_every:
            thermo = torch.empty((nsteps // thermo_every, 3), dtype=torch.float64, device=self.device)
        L.md_step_every(self.params, self.ws, nsteps, rebuild_every, thermo_every if thermo is not None else 0, thermo)
        return thermo

    def step_list(self, nsteps: int, rebuild_every: int, thermo_every: int = 0):
        """md_step_list: as step_every, with pair lists recorded at each
        rebuild and walked in between (needs ``pair_lists=True``)."""
        thermo = None
        if thermo_every > 0 and nsteps >= thermo_every:
            thermo = torch.empty((nsteps // thermo_every, 3), dtype=torch.float64, device=self.device)
        L.md_step_list(self.params, self.ws, nsteps, rebuild_every, thermo_every if thermo is not None else 0, thermo)
        return thermo

    def step_nlist(self, nsteps: int, rebuild_every: int, thermo_every: int = 0):
        """md_step_nlist: as step_every, with per-atom neighbour lists written
        at each rebuild and walked in between (needs ``atom_lists=True``)."""
        thermo = None
        if thermo_every > 0 and nsteps >= thermo_every:
            thermo = torch.empty((nsteps // thermo_every, 3), dtype=torch.float64, device=self.device)
        L.md_step_nlist(self.params, self.ws, nsteps, rebuild_every, thermo_every if thermo is not None else 0, thermo)
        return thermo

    def energy(self) -> torch.Tensor:
        out = torch.empty(3, dtype=torch.float64, device=self.device)
        L.md_energy_virial(self.params, self.ws, out)
        return out

    def thermo(self) -> torch.Tensor:
        """(U, K, W, T, P) of the current state, FP64 on the device: T =
        2K / (3N - 3), P = (2K + W) / (3V) (md_thermo)."""
        out = torch.empty(5, dtype=torch.float64, device=self.device)
        L.md_thermo(self.params, self.ws, out)
        return out

    def state(self):
        pos = torch.empty((self.n, 4), dtype=torch.float32, device=self.device)
        vel = torch.empty((self.n, 4), dtype=torch.float32, device=self.device)
        L.md_get_state(self.params, self.ws, pos, vel)
        return pos, vel

    def neighbors(self, max_per_atom: int = 128, lists: str | None = None):
        """Neighbour rows as the force kernel's walk accepts them; ``lists``:
        None screens against r_c (md_neighbors), "record" screens against the
        list radius and keeps the words, "kept" walks the words kept last
        (md_neighbors_lists)."""
        counts = torch.empty(self.n, dtype=torch.int32, device=self.device)
        idx = torch.full((self.n * max_per_atom,), -1, dtype=torch.int32, device=self.device)
        if lists is None:
            L.md_neighbors(self.params, self.ws, counts, idx, max_per_atom)
        else:
            L.md_neighbors_lists(self.params, self.ws, counts, idx, max_per_atom, lists == "record")
        return counts, idx.view(self.n, max_per_atom)

    def cell_lists(self):
        start = torch.empty(self.n_cells + 1, dtype=torch.int32, device=self.device)
        order = torch.empty(self.n, dtype=torch.int32, device=self.device)
        L.md_cell_lists(self.params, self.ws, start, order)
        return start, order

    def check(self, raise_on_error: bool = True) -> int:
        return L.md_check(self.ws, raise_on_error=raise_on_error)
