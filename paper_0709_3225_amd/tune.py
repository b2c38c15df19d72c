"""Autotuner for batches of replicas and single systems.

The only geometric choice the method leaves open is the cell side: section 3
asks for cells of side at least r_c, and section 3.2 takes the finest such
grid, n_c = int(L / r_c). Coarser grids stage more candidates per home cell
but fill more lanes of the one-wavefront-per-cell kernel; which wins depends
on the occupancy of the cells, so it is measured, not modelled. The force
pass may also split a cell's candidates over two or four wavefronts
(md_params.waves_per_cell), which pays only where the grid has too few cells
to fill the GPU, and its LDS tile (md_params.tile_cap) trades passes over
large neighbourhoods against wavefronts per CU; tune_system measures all
three knobs on one system, and tune_batch, given candidate wavefront counts
and tile offsets, per replica-size bucket of a batch.

Replicas are grouped into size buckets (their default grid and its mean
occupancy). For each bucket the tuner times batched steps of a probe made of
copies of one member replica's own state, once per candidate grid (the
default, up to ``extra`` coarser ones, and the grid sized for about 14 atoms
per cell), and keeps a coarser grid only if it is faster per atom-step by at
least ``min_gain``. The result is a per-replica
``cell_min`` for the replica table (0 keeps the default grid).

This module is host logic: every step it times runs in the library's kernels
through the C-ABI.
"""
from __future__ import annotations

import math
import time

import torch

from . import _lib as L
from .batch import BatchedLJ


def grid_options(n: int, box: float, *, rc_over_sigma: float = 2.5, sigma: float = 1.0, extra: int = 1,
                 max_occupancy: float = 48.0, target: float = 14.0):
    """Candidate cell grids of one replica as (cells_per_dim, cell_min): the
    default grid of md_cell_grid (cell_min 0), up to ``extra`` coarser ones,
    and the grid whose cells hold about ``target`` atoms (sparse systems,
    where the default cells hold one or two), each with at least 2 cells per
    dimension and at most ``max_occupancy`` atoms per cell on average. A
    coarser grid n_c is selected by cell_min = L / (n_c + 1/2), and
    md_cell_grid confirms it."""
    from .system import occupancy_cell_min

    base = dict(rc_over_sigma=rc_over_sigma, sigma=sigma)
    nc0, _ = L.md_cell_grid(L.make_params(n, box, **base))
    wanted = [nc0 - k for k in range(1, extra + 1)]
    nc_occ, _ = L.md_cell_grid(L.make_params(n, box, cell_min=occupancy_cell_min(n, box, rc_over_sigma * sigma,
                                                                                   target), **base))
    wanted.append(nc_occ)
    out = [(nc0, 0.0)]
    for nc in wanted:
        if nc >= nc0 or nc < 2 or n / nc ** 3 > max_occupancy or any(nc == o for o, _ in out):
            continue
        cm = float(box) / (nc + 0.5)
        got, _ = L.md_cell_grid(L.make_params(n, box, cell_min=cm, **base))
        if got == nc:
            out.append((nc, cm))
    return out


def bucket_key(n: int, nc0: int):
    """Replica-size bucket: the default grid and its mean occupancy, rounded."""
    return nc0, int(round(n / nc0 ** 3))


def _time_probe(n, box, cell_min, p4, v4, copies, steps, warmup, repeats, shared, stream, waves=0, tile=0):
    """Seconds per atom-step of a probe batch: the fastest of ``repeats``
    timed runs of ``steps`` steps after ``warmup`` untimed ones."""
    table = [(n, box, cell_min, waves, tile)] * copies
    b = BatchedLJ(table, **shared)
    pos = p4.repeat(copies, 1).contiguous()
    vel = v4.repeat(copies, 1).contiguous()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(repeats)]
    # the copies above (and the workspace) were made on the caller's stream
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        b.load(pos, vel)
        b.step(warmup)
        for e0, e1 in events:
            e0.record(stream)
            b.step(steps)
            e1.record(stream)
    stream.synchronize()
    b.check()
    best = min(e0.elapsed_time(e1) for e0, e1 in events) / 1e3
    return best / (steps * n * copies)


def _offset_tile(n, box, cell_min, offset, shared):
    """md_params.tile_cap for the formula's tile of this replica plus offset
    atoms (0: the formula itself, or an offset that leaves [128, 2048])."""
    if offset == 0:
        return 0
    q = {k: v for k, v in shared.items() if k in ("epsilon", "sigma", "mass", "rc_over_sigma", "dt", "shift_mode")}
    t = L.md_tile_capacity(L.make_params(n, box, cell_min=cell_min, **q)) + int(offset)
    return t if 128 <= t <= 2048 and t % 64 == 0 else 0


def tune_batch(replicas, pos4: torch.Tensor, vel4: torch.Tensor, *, epsilon=1.0, sigma=1.0, mass=1.0,
               rc_over_sigma=2.5, dt=0.005, shift_mode=0, extra=1, waves=(1,), tiles=(0,), min_atoms=131072,
               steps=10, warmup=3, repeats=3, min_gain=0.03):
    """Pick a cell grid, and optionally the wavefronts per cell and the LDS
    tile, per replica-size bucket.

    replicas: sequence of (n, box); pos4/vel4: the batch's concatenated float4
    state on the GPU (each bucket's probe copies one member's own atoms).
    Candidates per bucket are its grid_options x ``waves`` x ``tiles`` (tile
    offsets in atoms from each grid's formula tile, 0 being the formula); the
    defaults search the grid only. A candidate replaces the default (default
    grid, the first wavefront count, the formula's tile) only if it is faster
    per atom-step by ``min_gain``, and its tile replaces the formula's only
    if it also beats that on the same grid and wavefront count by
    ``min_gain``. Returns (cell_mins, report): cell_mins[b] goes into replica
    b's table entry; report["table"] holds the full entries (n, box,
    cell_min, waves_per_cell, tile_cap) for BatchedLJ (waves_per_cell 0 when
    only one count was tried); report["buckets"] lists, per bucket, the
    candidates with their measured seconds per atom-step and the choice."""
    shared = dict(epsilon=epsilon, sigma=sigma, mass=mass, rc_over_sigma=rc_over_sigma, dt=dt,
                  shift_mode=shift_mode)
    reps = [(int(n), float(box)) for n, box, *_ in replicas]
    offsets = [0]
    for n, _ in reps:
        offsets.append(offsets[-1] + n)
    options = [grid_options(n, box, rc_over_sigma=rc_over_sigma, sigma=sigma, extra=extra) for n, box in reps]
    buckets = {}
    for i, (n, _) in enumerate(reps):
        buckets.setdefault(bucket_key(n, options[i][0][0]), []).append(i)
    stream = torch.cuda.Stream()
    t_start = time.perf_counter()
    cell_mins = [0.0] * len(reps)
    table = [(n, box, 0.0, 0, 0) for n, box in reps]
    report = []
    for key, members in sorted(buckets.items()):
        i = members[0]
        n, box = reps[i]
        p4 = pos4[offsets[i]:offsets[i + 1]]
        v4 = vel4[offsets[i]:offsets[i + 1]]
        copies = max(1, math.ceil(min_atoms / n))
        tried = []
        for nc, cm in options[i]:
            for wv in waves:
                seen = set()
                for off in tiles:
                    tc = _offset_tile(n, box, cm, off, shared)
                    if tc in seen:
                        continue
                    seen.add(tc)
                    t = _time_probe(n, box, cm, p4, v4, copies, steps, warmup, repeats, shared, stream,
                                    wv if len(waves) > 1 else 0, tc)
                    tried.append({"cells_per_dim": nc, "cell_min": cm, "waves_per_cell": wv,
                                  "tile_offset": off if tc else 0, "tile_cap": tc, "s_per_atom_step": t})
        best = tried[0]
        for cand in tried[1:]:
            if cand["s_per_atom_step"] < best["s_per_atom_step"] * (1.0 - min_gain):
                best = cand
        same = [t for t in tried if t["cell_min"] == best["cell_min"] and t["waves_per_cell"] == best["waves_per_cell"]
                and t["tile_cap"] == 0]
        if same and best["s_per_atom_step"] >= same[0]["s_per_atom_step"] * (1.0 - min_gain):
            best = same[0]
        for j in members:
            # members share the default grid; the chosen coarser grid is
            # re-derived for each (same n_c, its own box), and the tile from
            # each member's own formula tile and the chosen offset
            nj, bj = reps[j]
            cmj = 0.0
            if best["cell_min"] != 0.0:
                for nc, cm in options[j]:
                    if nc == best["cells_per_dim"]:
                        cmj = cm
            cell_mins[j] = cmj
            table[j] = (nj, bj, cmj, best["waves_per_cell"] if len(waves) > 1 else 0,
                        _offset_tile(nj, bj, cmj, best["tile_offset"], shared))
        report.append({"bucket": {"cells_per_dim": key[0], "atoms_per_cell": key[1]}, "replicas": len(members),
                       "tried": tried, "chosen_cells_per_dim": best["cells_per_dim"],
                       "chosen_waves_per_cell": best["waves_per_cell"], "chosen_tile_offset": best["tile_offset"]})
    return cell_mins, {"buckets": report, "table": table, "seconds": time.perf_counter() - t_start}


def tune_cell_min(n: int, box: float, pos4: torch.Tensor, vel4: torch.Tensor, **kw):
    """The tuner on one system (for LJSystem): returns (cell_min, report)."""
    cms, report = tune_batch([(n, box)], pos4, vel4, **kw)
    return cms[0], report


def tile_options(p: L.MDParams, offsets=(0, 128, -64)):
    """Candidate LDS tiles of one system: md_params.tile_cap values for the
    formula's tile T (0) and for T + offset, kept within [128, 2048] and
    distinct."""
    t0 = L.md_tile_capacity(p)
    out = []
    for off in offsets:
        t = 0 if off == 0 else t0 + int(off)
        if t != 0 and (t < 128 or t > 2048 or t % 64 != 0 or t == t0):
            continue
        if t not in out:
            out.append(t)
    return out


def tune_system(n: int, box: float, pos4: torch.Tensor, vel4: torch.Tensor, *, epsilon=1.0, sigma=1.0, mass=1.0,
                rc_over_sigma=2.5, dt=0.005, shift_mode=0, extra=1, waves=(1, 2, 4), tiles=(0, 128, -64), steps=20,
                warmup=3, repeats=3, min_gain=0.03):
    """Pick the cell grid, the wavefronts per cell and the LDS tile of one
    system by timing md_step on the system itself (not on copies: a small
    system's grid holds too few cells to fill the GPU with one wavefront
    each, which is where several wavefronts per cell pay). Candidates are
    grid_options x waves x tile_options (tile offsets in atoms from the
    formula's tile of each grid, 0 being the formula); a candidate replaces
    the default (default grid, one wavefront, the formula's tile) only if it
    is faster per step by at least ``min_gain``, and its tile replaces the
    formula's only if it also beats that on the same grid and wavefront count
    by ``min_gain``. Returns
    (cell_min, waves_per_cell, tile_cap, report); tile_cap 0 is the formula."""
    from .system import LJSystem

    shared = dict(epsilon=epsilon, sigma=sigma, mass=mass, rc_over_sigma=rc_over_sigma, dt=dt, shift_mode=shift_mode)
    t_start = time.perf_counter()
    stream = torch.cuda.Stream()
    tried = []
    for nc, cm in grid_options(n, box, rc_over_sigma=rc_over_sigma, sigma=sigma, extra=extra):
        p = L.make_params(n, box, cell_min=cm, **shared)
        for wv in waves:
            for tc in tile_options(p, tiles):
                s = LJSystem(n, box, cell_min=cm, waves_per_cell=wv, tile_cap=tc, **shared)
                events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                          for _ in range(repeats)]
                # the workspace was allocated on the caller's stream
                stream.wait_stream(torch.cuda.current_stream())
                with torch.cuda.stream(stream):
                    s.load(pos4, vel4)
                    s.step(warmup)
                    for e0, e1 in events:
                        e0.record(stream)
                        s.step(steps)
                        e1.record(stream)
                stream.synchronize()
                s.check()
                best_t = min(e0.elapsed_time(e1) for e0, e1 in events) / 1e3 / steps
                tried.append({"cells_per_dim": nc, "cell_min": cm, "waves_per_cell": wv, "tile_cap": tc,
                              "tile_atoms": L.md_tile_capacity(s.params), "s_per_step": best_t})
    best = min(tried, key=lambda t: t["s_per_step"])
    if best["s_per_step"] >= tried[0]["s_per_step"] * (1.0 - min_gain):
        best = tried[0]
    # the tile moves off the formula's only if that beats the formula's tile on
    # the same grid and wavefront count by min_gain as well
    same = [t for t in tried if t["cell_min"] == best["cell_min"] and t["waves_per_cell"] == best["waves_per_cell"]
            and t["tile_cap"] == 0]
    if same and best["s_per_step"] >= same[0]["s_per_step"] * (1.0 - min_gain):
        best = same[0]
    report = {"tried": tried,
              "chosen": {k: best[k] for k in ("cells_per_dim", "cell_min", "waves_per_cell", "tile_cap", "tile_atoms")},
              "seconds": time.perf_counter() - t_start}
    return best["cell_min"], best["waves_per_cell"], best["tile_cap"], report
