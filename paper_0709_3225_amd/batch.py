"""Batches of independent LJ replicas on one GPU.

`BatchedLJ` owns one workspace for many replicas of different size and
density (shared epsilon, sigma, mass, cutoff and dt) and forwards to the
md_batch_* entry points of the C-ABI. `run_graph` captures a whole multi-step
run into one graph with md_batch_graph_create and starts it with a single
md_graph_launch; each replica follows exactly the arithmetic of md_step on
that system alone, so its results are bitwise those of a solo run.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L


class BatchedLJ:
    def __init__(self, replicas, *, epsilon=1.0, sigma=1.0, mass=1.0, rc_over_sigma=2.5, dt=0.005, cell_min=0.0,
                 shift_mode=0, waves_per_cell=0, device="cuda"):
        """replicas: sequence of (n, box[, cell_min[, waves_per_cell[,
        tile_cap]]]); a replica's nonzero cell_min and waves_per_cell replace
        the shared ones and its nonzero tile_cap the formula's tile
        (tune.tune_batch picks them)."""
        self.replicas = [(int(r[0]), float(r[1]), float(r[2]) if len(r) > 2 else 0.0,
                          int(r[3]) if len(r) > 3 else 0, int(r[4]) if len(r) > 4 else 0) for r in replicas]
        self.count = len(self.replicas)
        self.table = L.replica_table(self.replicas)
        self.params = L.make_params(1, 1.0, epsilon, sigma, mass, rc_over_sigma, dt, cell_min, shift_mode, 0,
                                    waves_per_cell)
        self.nbytes = int(L.lib().md_batch_workspace_bytes(ctypes.byref(self.params), self.table, self.count))
        if self.nbytes == 0:
            # reproduce the validation error with its message
            L._check(L.lib().md_batch_forces(ctypes.byref(self.params), self.table, self.count, None, 0, None, None))
            raise L.MDError(L.MD_ERR_ARG, "invalid batch")
        self.device = torch.device(device)
        self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        self.n_total = sum(r[0] for r in self.replicas)
        self.offsets = [0]
        for r in self.replicas:
            self.offsets.append(self.offsets[-1] + r[0])

    def _args(self):
        wp, wn = L._ws(self.ws)
        return ctypes.byref(self.params), self.table, self.count, wp, wn

    def _vec(self, t, name):
        return L._ptr(t, name, torch.float32, (self.n_total, 4))

    def load(self, pos4, vel4=None, forces=True, stream=None):
        L._check(L.lib().md_batch_build(*self._args(), self._vec(pos4, "pos4"),
                                        None if vel4 is None else self._vec(vel4, "vel4"), L._stream(stream)))
        if forces:
            self.forces(stream=stream)

    def forces(self, out=None, stream=None):
        L._check(L.lib().md_batch_forces(*self._args(), None if out is None else self._vec(out, "force4"),
                                         L._stream(stream)))
        return out

    def step(self, nsteps, thermo_every=0, stream=None):
        thermo = None
        tp = None
        if thermo_every > 0 and nsteps >= thermo_every:
            thermo = torch.empty((nsteps // thermo_every, self.count, 3), dtype=torch.float64, device=self.device)
            tp = L._ptr(thermo, "thermo", torch.float64)
        L._check(L.lib().md_batch_step(*self._args(), int(nsteps), int(thermo_every) if tp else 0, tp,
                                       L._stream(stream)))
        return thermo

    def energy(self, stream=None):
        out = torch.empty((self.count, 3), dtype=torch.float64, device=self.device)
        L._check(L.lib().md_batch_energy_virial(*self._args(), L._ptr(out, "out", torch.float64), L._stream(stream)))
        return out

    def state(self, stream=None):
        pos = torch.empty((self.n_total, 4), dtype=torch.float32, device=self.device)
        vel = torch.empty((self.n_total, 4), dtype=torch.float32, device=self.device)
        L._check(L.lib().md_batch_get_state(*self._args(), self._vec(pos, "pos4"), self._vec(vel, "vel4"),
                                            L._stream(stream)))
        return pos, vel

    def make_graph(self, nsteps, thermo_every=0, stream=None):
        """Capture nsteps batched steps into a graph on a non-null stream.
        Returns (graph handle, thermo tensor or None)."""
        if stream is None:
            stream = torch.cuda.current_stream()
        thermo = None
        tp = None
        if thermo_every > 0 and nsteps >= thermo_every:
            thermo = torch.empty((nsteps // thermo_every, self.count, 3), dtype=torch.float64, device=self.device)
            tp = L._ptr(thermo, "thermo", torch.float64)
        g = ctypes.c_void_p()
        L._check(L.lib().md_batch_graph_create(*self._args(), int(nsteps), int(thermo_every) if tp else 0, tp,
                                               L._stream(stream), ctypes.byref(g)))
        return BatchGraph(g, self), thermo

    def check(self, raise_on_error=True):
        return L.md_check(self.ws, raise_on_error=raise_on_error)


class BatchGraph:
    """Owner of an instantiated batched-run graph (keeps the batch alive)."""

    def __init__(self, handle, batch):
        self.handle = handle
        self.batch = batch

    def launch(self, stream=None):
        L._check(L.lib().md_graph_launch(self.handle, L._stream(stream)))

    def close(self):
        if self.handle:
            L._check(L.lib().md_graph_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown: nothing left to release into
            pass
