"""Throughput benchmark of the LJ cell-list MD step on one MI355X.

One step = velocity-Verlet half kick + drift + wrap + cell-list rebuild
(histogram, scan, scatter, in-cell order) + LJ forces over the 27-cell
neighbourhood + half kick, with FP64 energy/virial/kinetic reductions every
--thermo-every steps. Default workload: N = 256000 LJ fluid (40^3 FCC start,
rho = 0.8442, T* = 0.722, r_c = 2.5 sigma, dt = 0.005), synthetic.

Prints one JSON line with the whole-job atom-steps/s, the roofline of the
force kernel (timed live with HIP events on the launch stream) and the FP64
oracle's throughput on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "atom-steps/s LJ cell-list FP32 + % FP32 peak; batched & adjoint vs plain"
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X: 256 CUs x 2.4 GHz x 256 FP32 flop/clk
FP32_MATRIX_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix-core peak
FLOP_PER_CANDIDATE = 8           # displacement (3) + r^2 (5)
FLOP_PER_ACCEPTED = 17           # rsqrt, powers, shifted magnitude, 3 accumulating FMAs
# Hessian-vector product pass of the adjoint, per accepted pair: powers and
# phi/r (12), phi' and B = (phi' - g)/r^2 (6), dphi/dsigma / r (7), w_i - w_j (3),
# d.(w_i - w_j) (5), B times it (1), J accumulation (12), force for d/d eps (6),
# d.w_i and the sigma term (7)
FLOP_PER_ACCEPTED_HVP = 59
MFMA_MIN_HOME, MFMA_MAX_HOME = 11, 16  # home-atom chunks screened on the matrix cores


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="lj256k")
    ap.add_argument("--thermo-every", type=int, default=100)
    ap.add_argument("--force-reps", type=int, default=200, help="md_forces launches timed for the roofline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device-to-device copy of this size (HBM counter calibration)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint throughput leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-replica throughput leg")
    ap.add_argument("--no-widened", action="store_true", help="skip the density-axis, WCA and skin legs")
    ap.add_argument("--only", choices=("adjoint", "batched", "neighbor_list"),
                    help="run only this leg and print its JSON (for kernel traces of one leg)")
    return ap.parse_args()


def batched_leg(torch, nsteps=200, seq_steps=20):
    """512 replicas (N = 4 n^3, n uniform in [5, 20], rho in [0.70, 0.95],
    T* in [0.7, 1.5]) advanced nsteps steps by one launch of a captured graph,
    against the same replicas run one after another with md_step."""
    import numpy as np

    import ljsynth
    from paper_0709_3225_amd import BatchedLJ, LJSystem, tune_batch

    ws = ljsynth.batched_replicas(512, 4)
    states = [ljsynth.make_state(w) for w in ws]
    table = [(w.n, box) for w, (_, _, box) in zip(ws, states)]
    pos = torch.from_numpy(np.concatenate([s[0] for s in states])).cuda()
    vel = torch.from_numpy(np.concatenate([s[1] for s in states])).cuda()

    def graph_time(b):
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            b.load(pos, vel)
            graph, _ = b.make_graph(nsteps)
            graph.launch()  # warm
        stream.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        graph.launch(stream)
        e1.record(stream)
        stream.synchronize()
        t = max(time.perf_counter() - t0, e0.elapsed_time(e1) / 1e3)
        graph.close()
        b.check()
        return t

    b = BatchedLJ(table)
    t_batch = graph_time(b)
    # cell grid, wavefronts per cell and LDS tile picked per replica-size
    # bucket by measurement, same run
    cms, rep = tune_batch(table, pos, vel, waves=(1, 4), tiles=(0, -64))
    bt = BatchedLJ(rep["table"])
    t_tuned = graph_time(bt)
    del bt
    # the same replicas one after another (md_step per replica)
    solos = []
    for (n, box), (p4, v4, _) in zip(table, states):
        s = LJSystem(n, box)
        s.load(torch.from_numpy(p4).cuda(), torch.from_numpy(v4).cuda())
        solos.append(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in solos:
        s.step(seq_steps)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    for s in solos[:4]:
        s.check()
    ntot = b.n_total
    value = ntot * nsteps / t_batch
    seq = ntot * seq_steps / t_seq
    return {
        "workload": f"512 replicas, N = 4 n^3 with n uniform in [5, 20] (total {ntot} atoms), rho in [0.70, 0.95], "
                    f"T* in [0.7, 1.5], {nsteps} steps in one graph launch",
        "value": value, "unit": "atom-steps/s", "ms_per_launch": t_batch * 1e3,
        "sequential_value": seq, "ratio_vs_sequential": value / seq,
        "autotuned": {"value": ntot * nsteps / t_tuned, "ms_per_launch": t_tuned * 1e3,
                      "tune_seconds": rep["seconds"], "buckets": len(rep["buckets"]),
                      "knobs": "cell side x waves per cell (1, 4) x LDS tile (formula, -64 atoms) per bucket",
                      "replicas_on_coarser_grids": sum(1 for cm in cms if cm > 0.0),
                      "replicas_on_4_waves": sum(1 for r in rep["table"] if r[3] == 4),
                      "replicas_on_smaller_tiles": sum(1 for r in rep["table"] if r[4] != 0)},
    }


def _timed_gradient(torch, x, v, box, nsteps, **kw):
    from paper_0709_3225_amd import trajectory_gradients

    trajectory_gradients(x, v, box, nsteps=20, every=20, **kw)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = trajectory_gradients(x, v, box, nsteps=nsteps, every=20, **kw)
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def adjoint_leg(torch):
    """Forward + backward of L = K_T/N + W_T/(3V) through 200 Verlet steps at
    N = 32000 (checkpoints every 20 steps, each segment recomputed on a second
    stream while the one after it is swept), against plain md_step at the same
    size. Both in atom-steps/s (N x 200 / time). Also: the same checkpointed
    gradient on one stream, and with every state kept in the forward (no
    recomputation)."""
    import ljsynth
    from paper_0709_3225_amd import LJSystem

    w = ljsynth.WORKLOADS["lj32k_adjoint"]
    pos4, vel4, box = ljsynth.make_state(w)
    x, v = torch.from_numpy(pos4).cuda(), torch.from_numpy(vel4).cuda()
    (loss, gr, gv, ge, gs), t_adj = _timed_gradient(torch, x, v, box, w.steps)
    _, t_seq = _timed_gradient(torch, x, v, box, w.steps, overlap=False)
    _, t_kept = _timed_gradient(torch, x, v, box, w.steps, keep_path=True)
    s = LJSystem(w.n, box, dt=w.dt)
    s.load(x, v)
    s.step(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(w.steps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    s.check()
    work = w.n * w.steps
    plain = work / t_plain
    hvp = hvp_roofline(s, torch)
    # the same gradient at the headline size (N = 256,000), where the grid
    # fills the chip: context for how the ratio depends on the size
    wl = ljsynth.WORKLOADS["lj256k"]
    pos4, vel4, boxl = ljsynth.make_state(wl)
    xl, vl = torch.from_numpy(pos4).cuda(), torch.from_numpy(vel4).cuda()
    _, t_l = _timed_gradient(torch, xl, vl, boxl, w.steps)
    _, t_l_seq = _timed_gradient(torch, xl, vl, boxl, w.steps, overlap=False)
    _, t_l_kept = _timed_gradient(torch, xl, vl, boxl, w.steps, keep_path=True)
    work_l = wl.n * w.steps
    return {
        "workload": f"{w.name}: N={w.n}, rho={w.density}, T*={w.temperature}, {w.steps} steps, checkpoints every 20, "
                    "loss K_T/N + W_T/(3V), gradients w.r.t. r0, v0, eps, sigma",
        "value": work / t_adj, "unit": "atom-steps/s (forward + backward)", "plain_value": plain,
        "ratio_vs_plain": work / t_adj / plain, "loss": loss, "dL_deps": ge, "dL_dsigma": gs,
        "one_stream": {"value": work / t_seq, "ratio_vs_plain": work / t_seq / plain},
        "kept_path": {"value": work / t_kept, "ratio_vs_plain": work / t_kept / plain,
                      "path_bytes": w.steps * (16 * w.n + 4 * (s.cells_per_dim ** 3 + 1))},
        "value_at_256k": work_l / t_l,
        "at_256k_one_stream": work_l / t_l_seq,
        "at_256k_kept_path": work_l / t_l_kept,
        "hvp_roofline": hvp,
        "hvp_roofline_at_256k": hvp_roofline(_loaded(torch, wl), torch),
    }


def _loaded(torch, w):
    import ljsynth
    from paper_0709_3225_amd import LJSystem

    pos4, vel4, box = ljsynth.make_state(w)
    s = LJSystem(w.n, box, dt=w.dt)
    s.load(torch.from_numpy(pos4).cuda(), torch.from_numpy(vel4).cuda())
    s.step(20)
    return s


def hvp_roofline(s, torch, reps=100):
    """The Hessian-vector product pass of the adjoint (k_pair_pass<OP_ADJ>,
    one md_adjoint_kick: the pair pass plus a gather of the vector into cell
    order) on the system's current cells: HIP events over reps calls on the
    launch stream, algorithmic flops split as for the force kernel (59 per
    accepted pair)."""
    from paper_0709_3225_amd import _lib as L

    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    w4 = torch.randn((s.n, 4), generator=g, device="cuda", dtype=torch.float32)
    lam = torch.zeros((s.n, 4), device="cuda", dtype=torch.float32)
    stream = torch.cuda.current_stream()
    L.md_adjoint_kick(s.params, s.ws, w4, lam, None, 1.0)  # warm
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        L.md_adjoint_kick(s.params, s.ws, w4, lam, None, 1.0)
    e1.record(stream)
    torch.cuda.synchronize()
    s.check()
    us = e0.elapsed_time(e1) * 1e3 / reps
    return {"kernel": "k_pair_pass<OP_ADJ> (md_adjoint_kick: pair pass + gather of n float4)", "n": s.n,
            **alu_roofline(pair_counts(s, torch), FLOP_PER_ACCEPTED_HVP, us)}


def _timed_steps(s, nsteps, torch, every=0):
    """Seconds for nsteps of md_step (or md_step_every with rebuilds every
    `every` steps): the larger of HIP-event and wall time."""
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    if every:
        s.step_every(nsteps, every)
    else:
        s.step(nsteps)
    e1.record(stream)
    torch.cuda.synchronize()
    return max(time.perf_counter() - t0, e0.elapsed_time(e1) / 1e3)


def _widened_point(torch, w, cell_min, nsteps, warm):
    import ljsynth
    from paper_0709_3225_amd import LJSystem

    pos4, vel4, box = ljsynth.make_state(w)
    s = LJSystem(w.n, box, rc_over_sigma=w.rc_over_sigma, shift_mode=w.shift_mode, dt=w.dt, cell_min=cell_min)
    s.load(torch.from_numpy(pos4).cuda(), torch.from_numpy(vel4).cuda())
    s.step(warm)
    t = _timed_steps(s, nsteps, torch)
    s.check()
    return {"cells_per_dim": s.cells_per_dim, "cell_side": round(s.cell_side, 4),
            "atoms_per_cell": round(w.n / s.n_cells, 2), "value": w.n * nsteps / t,
            "us_per_step": t * 1e6 / nsteps}


def full_size_leg(torch, nsteps=100, warm=20):
    """The N = 2,048,000 configuration (80^3 FCC, rho = 0.8442, T* = 1.0) on
    one GPU: md_step atom-steps/s with the cell list rebuilt every step (its
    grid of 148,877 cells takes the tiled block scan)."""
    import ljsynth

    w = ljsynth.WORKLOADS["lj2m"]
    pt = _widened_point(torch, w, 0.0, nsteps, warm)
    pt["workload"] = (f"{w.name}: LJ N={w.n} (80^3 FCC start), rho={w.density}, T*={w.temperature}, rc=2.5 sigma "
                      f"force-shifted, dt={w.dt}, {nsteps} steps after {warm}, cell list rebuilt every step")
    pt["unit"] = "atom-steps/s"
    return pt


def density_leg(torch, nsteps=100, warm=20):
    """LJ (r_c = 2.5 sigma) at N = 256,000 along the density axis of the
    paper's cell-list measurements (section 3.2): md_step atom-steps/s with the
    paper's cells (side >= r_c), with cells sized for about 14 atoms, and with
    the grid the autotuner picks by measurement."""
    import ljsynth
    from paper_0709_3225_amd import occupancy_cell_min, tune_cell_min

    points = []
    for rho in ljsynth.DENSITY_SWEEP:
        w = ljsynth.sweep_workload(rho)
        box = ljsynth.box_length(w.n, rho)
        for cells, cm in (("paper", 0.0), ("occupancy", occupancy_cell_min(w.n, box, w.rc_over_sigma))):
            pt = _widened_point(torch, w, cm, nsteps, warm)
            pt.update({"rho": rho, "cells": cells})
            points.append(pt)
        pos4, vel4, _ = ljsynth.make_state(w)
        cm, rep = tune_cell_min(w.n, box, torch.from_numpy(pos4).cuda(), torch.from_numpy(vel4).cuda(),
                                rc_over_sigma=w.rc_over_sigma, shift_mode=w.shift_mode, dt=w.dt)
        pt = _widened_point(torch, w, cm, nsteps, warm)
        pt.update({"rho": rho, "cells": "tuned", "tune_seconds": round(rep["seconds"], 3)})
        points.append(pt)
    return {"workload": "LJ N=256000 (40^3 FCC start), T*=0.722, rc=2.5 sigma force-shifted, dt=0.005, "
                        f"{nsteps} steps after {warm}, rho in {list(ljsynth.DENSITY_SWEEP)}",
            "unit": "atom-steps/s", "points": points}


def wca_leg(torch, nsteps=100, warm=20):
    """WCA (LJ cut at 2^(1/6) sigma, shifted by eps) at N = 256,000,
    rho = 0.8442, T* = 0.722: md_step atom-steps/s with the paper's cells
    (side >= r_c) and with larger cells."""
    import ljsynth
    from paper_0709_3225_amd import occupancy_cell_min, tune_cell_min

    w = ljsynth.wca_workload()
    box = ljsynth.box_length(w.n, w.density)
    points = []
    for cells, cm in (("paper", 0.0), ("1.7", 1.7), ("2.1", 2.1),
                      ("occupancy", occupancy_cell_min(w.n, box, w.rc_over_sigma))):
        pt = _widened_point(torch, w, cm, nsteps, warm)
        pt["cells"] = cells
        points.append(pt)
    pos4, vel4, _ = ljsynth.make_state(w)
    cm, rep = tune_cell_min(w.n, box, torch.from_numpy(pos4).cuda(), torch.from_numpy(vel4).cuda(),
                            rc_over_sigma=w.rc_over_sigma, shift_mode=w.shift_mode, dt=w.dt)
    pt = _widened_point(torch, w, cm, nsteps, warm)
    pt.update({"cells": "tuned", "tune_seconds": round(rep["seconds"], 3)})
    points.append(pt)
    best = max(points, key=lambda p: p["value"])
    return {"workload": f"{w.name}: WCA N={w.n} (40^3 FCC start), rho={w.density}, T*={w.temperature}, "
                        f"rc=2^(1/6) sigma energy-shifted, dt={w.dt}, {nsteps} steps after {warm}",
            "unit": "atom-steps/s", "points": points, "best": best["cells"], "value": best["value"],
            "neighbor_list": wca_list_points(torch, w, box, nsteps, warm)}


def wca_list_points(torch, w, box, nsteps, warm):
    """The WCA workload with per-atom Verlet lists (md_step_nlist) of radius
    r_V = r_c + skin on the occupancy-sized cells: the lists hold about 15
    partners per atom against the 27 cells' 390 candidates. A point is valid
    without MD_DEV_SKIN (an atom moved by more than skin / 2 between
    rebuilds) or MD_DEV_NB_OVERFLOW."""
    from paper_0709_3225_amd import LJSystem, occupancy_cell_min
    import ljsynth

    pos4, vel4, _ = ljsynth.make_state(w)
    cm = occupancy_cell_min(w.n, box, w.rc_over_sigma)
    points = []
    for skin, every in ((0.3, 5), (0.3, 8), (0.5, 10), (0.5, 15)):
        s = LJSystem(w.n, box, rc_over_sigma=w.rc_over_sigma, shift_mode=w.shift_mode, dt=w.dt, cell_min=cm,
                     list_radius=w.rc_over_sigma + skin, atom_lists=True)
        s.load(torch.from_numpy(pos4).cuda(), torch.from_numpy(vel4).cuda())
        s.step(warm)
        s.step_nlist(every + 1, every)  # every kernel of the timed run once
        s.check(raise_on_error=False)
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        s.step_nlist(nsteps, every)
        e1.record(stream)
        torch.cuda.synchronize()
        t = max(time.perf_counter() - t0, e0.elapsed_time(e1) / 1e3)
        flags = s.check(raise_on_error=False)
        points.append({"list_radius": round(w.rc_over_sigma + skin, 4), "cells_per_dim": s.cells_per_dim,
                       "rebuild_every": every, "value": w.n * nsteps / t, "us_per_step": t * 1e6 / nsteps,
                       "valid": flags == 0})
    valid = [p for p in points if p["valid"]]
    best = max(valid, key=lambda p: p["value"]) if valid else None
    return {"points": points, "best": {k: best[k] for k in ("list_radius", "rebuild_every")} if best else None,
            "value": best["value"] if best else None}


def skin_leg(torch, nsteps=100, warm=20):
    """The headline workload with the cell lists rebuilt only every few steps
    (md_step_every; section 3.1): the skin is the grid's margin over r_c
    (cell_min picks the grid). A point is valid when no atom left its cell by
    half the skin (no MD_DEV_SKIN)."""
    import ljsynth
    from paper_0709_3225_amd import LJSystem

    w = ljsynth.WORKLOADS["lj256k"]
    pos4, vel4, box = ljsynth.make_state(w)
    points = []
    for cm, every in ((0.0, 1), (0.0, 2), (0.0, 3), (0.0, 4), (0.0, 6), (2.7, 4), (2.7, 8), (2.9, 10)):
        s = LJSystem(w.n, box, dt=w.dt, cell_min=cm)
        s.load(torch.from_numpy(pos4).cuda(), torch.from_numpy(vel4).cuda())
        s.step(warm)
        t = _timed_steps(s, nsteps, torch, every)
        flags = s.check(raise_on_error=False)
        points.append({"cells_per_dim": s.cells_per_dim, "skin": round(s.cell_side - w.rc_over_sigma, 4),
                       "rebuild_every": every, "value": w.n * nsteps / t, "us_per_step": t * 1e6 / nsteps,
                       "valid": flags == 0})
    best = max((p for p in points if p["valid"]), key=lambda p: p["value"])
    return {"workload": f"{w.name}: LJ N={w.n}, rho={w.density}, T*={w.temperature}, {nsteps} steps after {warm}, "
                        "cell lists rebuilt every k steps",
            "unit": "atom-steps/s", "points": points, "best": {k: best[k] for k in ("skin", "rebuild_every")},
            "value": best["value"]}


def pair_list_leg(torch, nsteps=100, warm=20, atom_lists=False):
    """The headline workload with pair lists (md_step_list): the force pass
    after each cell rebuild records every lane's candidates within the cell
    side, the passes in between walk them; the skin is the grid's margin over
    r_c. With atom_lists, md_step_nlist: the pass after each rebuild writes
    every atom's neighbour list, one lane per atom walks it in between. A
    point is valid when no atom moved by half the skin since the lists were
    recorded and no list overflowed (no MD_DEV_SKIN, MD_DEV_NB_OVERFLOW)."""
    import ljsynth
    from paper_0709_3225_amd import LJSystem

    w = ljsynth.WORKLOADS["lj256k"]
    pos4, vel4, box = ljsynth.make_state(w)
    points = []
    for cm, every in ((0.0, 2), (0.0, 3), (0.0, 4), (2.7, 6), (2.7, 10), (2.9, 10), (2.9, 15)):
        s = LJSystem(w.n, box, dt=w.dt, cell_min=cm, pair_lists=not atom_lists, atom_lists=atom_lists)
        s.load(torch.from_numpy(pos4).cuda(), torch.from_numpy(vel4).cuda())
        s.step(warm)
        run = s.step_nlist if atom_lists else s.step_list
        run(every + 1, every)  # every kernel of the timed run once
        s.check(raise_on_error=False)
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        run(nsteps, every)
        e1.record(stream)
        torch.cuda.synchronize()
        t = max(time.perf_counter() - t0, e0.elapsed_time(e1) / 1e3)
        flags = s.check(raise_on_error=False)
        points.append({"cells_per_dim": s.cells_per_dim, "skin": round(s.cell_side - w.rc_over_sigma, 4),
                       "rebuild_every": every, "value": w.n * nsteps / t, "us_per_step": t * 1e6 / nsteps,
                       "valid": flags == 0})
    valid = [p for p in points if p["valid"]]
    best = max(valid, key=lambda p: p["value"]) if valid else None
    kind = "per-atom neighbour lists written" if atom_lists else "pair lists recorded"
    return {"workload": f"{w.name}: LJ N={w.n}, rho={w.density}, T*={w.temperature}, {nsteps} steps after {warm}, "
                        f"{kind} at each cell rebuild (every k steps)",
            "unit": "atom-steps/s", "points": points,
            "best": {k: best[k] for k in ("skin", "rebuild_every")} if best else None,
            "value": best["value"] if best else None}


def pair_counts(sys_, torch, chunk=64):
    """Candidate pairs the 27-cell method tests on the current state, split
    into those screened on the VALU and those screened on the matrix cores
    (home-atom chunks of 11..16 atoms: a cell's atoms in chunks of `chunk`,
    each chunk against the whole neighbourhood; the kernels take chunks of
    64), and the accepted ordered pairs."""
    import numpy as np

    start, _ = sys_.cell_lists()
    cnt = np.diff(start.cpu().numpy().astype(np.int64))
    nc = sys_.cells_per_dim
    grid = cnt.reshape(nc, nc, nc)  # [z][y][x]
    hood = np.zeros_like(grid)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                hood += np.roll(grid, shift=(dz, dy, dx), axis=(0, 1, 2))
    candidates = int((grid * hood).sum())
    full = grid // chunk  # full chunks: on the matrix cores if 16 atoms, else (64) the VALU
    last = grid % chunk    # the last chunk
    mfma_home = np.where((last >= MFMA_MIN_HOME) & (last <= MFMA_MAX_HOME), last, 0)
    if chunk == MFMA_MAX_HOME:
        mfma_home = mfma_home + chunk * full
    mfma = int((mfma_home * hood).sum())
    counts, _ = sys_.neighbors(max_per_atom=1)  # counts only; rows truncate (flag cleared below)
    accepted = int(counts.sum().item())
    sys_.check(raise_on_error=False)
    return {"candidates": candidates, "valu_candidates": candidates - mfma, "mfma_candidates": mfma,
            "accepted_pairs": accepted}


def alu_roofline(pc, per_accepted, kernel_us):
    """Algorithmic flops of one cell-pair launch split by the unit that runs
    them: the VALU takes the screen of VALU-screened candidates (8 each) and
    every accepted pair's interaction; the matrix cores take the screen of the
    other candidates (8 each, as dot products). Each part over the launch's
    duration against its own FP32 peak."""
    t = kernel_us * 1e-6
    vec = FLOP_PER_CANDIDATE * pc["valu_candidates"] + per_accepted * pc["accepted_pairs"]
    mat = FLOP_PER_CANDIDATE * pc["mfma_candidates"]
    vec_tf = vec / t / 1e12
    mat_tf = mat / t / 1e12
    return {
        "bound": "alu",
        "achieved": vec_tf,
        "peak": FP32_VECTOR_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": vec_tf / FP32_VECTOR_PEAK_TFLOPS,
        "kernel_us": kernel_us,
        "vector_flops_per_launch": vec,
        "matrix": {"achieved": mat_tf, "peak": FP32_MATRIX_PEAK_TFLOPS, "unit": "TFLOP/s",
                   "frac": mat_tf / FP32_MATRIX_PEAK_TFLOPS, "flops_per_launch": mat},
        "all_flops_tflops": (vec + mat) / t / 1e12,
        **pc,
        # the interaction-only count: the candidate test and interaction of the
        # accepted pairs alone, the floor of any exact method, over the same time
        "interaction_only_tflops": (FLOP_PER_CANDIDATE + per_accepted) * pc["accepted_pairs"] / t / 1e12,
    }


FORCE_SOURCES = ("paper_0709_3225_amd/csrc/forces.hip", "paper_0709_3225_amd/csrc/cell_pairs.h",
                 "paper_0709_3225_amd/csrc/md_device.h",
                 "paper_0709_3225_amd/csrc/md_internal.h",
                 "paper_0709_3225_amd/build.py")  # the compiler flags shape the kernel too


def recorded_traffic(workload):
    """HBM bytes per force-kernel launch from the committed counter summary,
    or None if the force-kernel sources changed since the counters were taken
    (or no summary exists for this workload)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"k_forces_{workload}.md")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and line.split(":", 1)[0] in ("forces_source_sha256", "traffic_bytes_per_launch"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in FORCE_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if rec.get("forces_source_sha256") != h.hexdigest() or "traffic_bytes_per_launch" not in rec:
        return None
    return float(rec["traffic_bytes_per_launch"])


def cpu_cell_list(pos4, vel4, box, headline, steps=10):
    """Algorithm-matched CPU baseline: the same cell-list method in C with
    OpenMP threads and SIMD pair loops on the host cores (built here for this
    host's CPU), FP32 and FP64, on the same state; per-step time from runs of
    `steps` and 0 steps."""
    import cpu_cells

    cpu_cells.build(force=True, native=True)
    cores = cpu_cells.num_threads()
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    out = {"unit": "atom-steps/s", "cores": cores, "kind": "cell list (C, OpenMP threads, SIMD pair loops)", "cpu_model": model,
           "affinity_cpus": len(os.sched_getaffinity(0)),
           "sample": f"{steps} velocity-Verlet steps of the N={len(pos4)} state, cell list rebuilt every step"}

    def per_step_time(prec, k):
        t0 = time.perf_counter()
        cpu_cells.run(pos4, vel4, box, 0, precision=prec)
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        cpu_cells.run(pos4, vel4, box, k, precision=prec)
        return max(time.perf_counter() - t0 - t_setup, 1e-9) / k

    for prec in ("f32", "f64"):
        cpu_cells.run(pos4, vel4, box, 1, precision=prec)  # warm (threads, pages)
        t = per_step_time(prec, steps)
        v = len(pos4) / t
        out[prec] = {"value": v, "ms_per_step": t * 1e3, "gpu_ratio": headline / v}
    # one core, as the paper's speedups are quoted
    cpu_cells.set_threads(1)
    t = per_step_time("f32", 1)
    cpu_cells.set_threads(cores)
    v = len(pos4) / t
    out["f32_one_core"] = {"value": v, "ms_per_step": t * 1e3, "gpu_ratio": headline / v}
    return out


def cpu_baseline(pos4, box, target_s):
    """FP64 oracle: force rows of the same state (each row = all N partners),
    repeated until about target_s seconds; one oracle MD step costs one row
    per atom, so rows/s is its atom-steps/s."""
    import numpy as np

    import oracle

    oracle.build(force=False)
    p = oracle.params(box)
    n = len(pos4)
    rng = np.random.default_rng(123)
    rows_done, chunk = 0, 512
    t0 = time.perf_counter()
    while True:
        rows = rng.choice(n, size=chunk, replace=False)
        oracle.forces_rows(p, pos4, rows)
        rows_done += chunk
        el = time.perf_counter() - t0
        if el >= target_s:
            break
        if el < 0.25 * target_s:
            chunk = min(chunk * 2, 65536)
    return {
        "value": rows_done / el,
        "unit": "atom-steps/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{rows_done} uniformly sampled force rows of the N={n} state, each against all N atoms "
                  f"(FP64 brute force, minimum image), {el:.1f} s on the host; an oracle step costs one row per atom",
        "more": oracle_timings(pos4, box),
    }


_ONE_CORE_ROWS = """
import json, sys, time
import numpy as np
import oracle
pos4 = np.load(sys.argv[1])
p = oracle.params(float(sys.argv[2]))
rows = np.random.default_rng(7).choice(len(pos4), size=int(sys.argv[3]), replace=False)
oracle.forces_rows(p, pos4, rows[:8])
t0 = time.perf_counter()
oracle.forces_rows(p, pos4, rows)
print(json.dumps({"rows": len(rows), "seconds": time.perf_counter() - t0, "cores": oracle.num_threads()}))
"""


def oracle_timings(pos4, box):
    """The oracle's other timings: one core on rows of the same state (a
    child process with one OpenMP thread), the full 100 steps of the N = 4,000
    workload, and 4,096 force rows of the N = 2,048,000 state."""
    import subprocess
    import sys
    import tempfile

    import numpy as np

    import ljsynth
    import oracle

    out = {}
    with tempfile.TemporaryDirectory() as tmp:
        f = os.path.join(tmp, "pos4.npy")
        np.save(f, pos4)
        env = dict(os.environ, OMP_NUM_THREADS="1", PYTHONPATH=ROOT)
        res = subprocess.run([sys.executable, "-c", _ONE_CORE_ROWS, f, repr(float(box)), "1024"], env=env,
                             capture_output=True, text=True, timeout=300, check=True)
        r = json.loads(res.stdout.strip().splitlines()[-1])
        out["one_core"] = {"value": r["rows"] / r["seconds"], "unit": "atom-steps/s", "cores": r["cores"],
                           "sample": f"{r['rows']} force rows of the N={len(pos4)} state in {r['seconds']:.1f} s"}
    w = ljsynth.WORKLOADS["lj4k"]
    p4, v4, b4 = ljsynth.make_state(w)
    p = oracle.params(b4, dt=w.dt)
    t0 = time.perf_counter()
    oracle.run(p, p4, v4, w.steps)
    t = time.perf_counter() - t0
    out["lj4k_full_run"] = {"value": w.n * w.steps / t, "unit": "atom-steps/s", "cores": oracle.num_threads(),
                            "sample": f"all {w.steps} velocity-Verlet steps of N={w.n} in {t:.2f} s"}
    w = ljsynth.WORKLOADS["lj2m"]
    p2, _, b2 = ljsynth.make_state(w)
    rows = np.random.default_rng(9).choice(w.n, size=4096, replace=False)
    p = oracle.params(b2)
    t0 = time.perf_counter()
    oracle.forces_rows(p, p2, rows)
    t = time.perf_counter() - t0
    out["lj2m_rows"] = {"value": len(rows) / t, "unit": "atom-steps/s", "cores": oracle.num_threads(),
                        "sample": f"{len(rows)} force rows of the N={w.n} state in {t:.1f} s"}
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import ljsynth
    from paper_0709_3225_amd import LJSystem

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.only:
        legs = {"adjoint": adjoint_leg, "batched": batched_leg,
                "neighbor_list": lambda t: pair_list_leg(t, atom_lists=True)}
        leg = legs[args.only](torch)
        print(json.dumps({args.only: leg}), flush=True)
        return
    w = ljsynth.WORKLOADS[args.workload]
    pos4, vel4, box = ljsynth.make_state(w)
    s = LJSystem(w.n, box, epsilon=w.epsilon, sigma=w.sigma, mass=w.mass, rc_over_sigma=w.rc_over_sigma, dt=w.dt)
    s.load(torch.from_numpy(pos4).cuda(), torch.from_numpy(vel4).cuda())
    # the timed region's step kind (at least one FP64 thermo step) also in the
    # warm-up, so that every kernel it launches has run once before
    thermo_every = min(args.thermo_every, args.steps) if args.thermo_every > 0 else 0
    if args.warmup:
        s.step(args.warmup, thermo_every=min(thermo_every, args.warmup))
    s.check()
    stream = torch.cuda.current_stream()

    # ---- force kernel alone (md_forces without output = one kernel launch) on
    # the state the timed region starts from (recomputing its forces leaves the
    # state bitwise as it was): pair counts first, then the timed launches,
    # which run right before the timed region
    from paper_0709_3225_amd import md_forces

    pc = pair_counts(s, torch)
    reps = args.force_reps
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.forces()  # warm
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        md_forces(s.params, s.ws)
    e1.record(stream)
    thermo_buf = None
    if thermo_every > 0:
        thermo_buf = torch.empty((args.steps // thermo_every, 3), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    force_us = e0.elapsed_time(e1) * 1e3 / reps
    s.check()
    roof = alu_roofline(pc, FLOP_PER_ACCEPTED, force_us)

    # ---- timed region: K whole steps, at least one of them with the FP64
    # energy/virial/kinetic reduction
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    thermo = s.step(args.steps, thermo_every=thermo_every, thermo_out=thermo_buf)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_s = ev0.elapsed_time(ev1) / 1e3
    s.check()
    elapsed = max(wall, gpu_s)
    value = w.n * args.steps / elapsed

    e_th = None
    if thermo is not None:
        th = thermo.cpu().numpy()
        e_th = {"U_per_atom": float(th[-1, 0] / w.n), "K_per_atom": float(th[-1, 1] / w.n),
                "W_per_atom": float(th[-1, 2] / w.n)}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: LJ fluid N={w.n} ({w.n_fcc}^3 FCC start), rho={w.density}, T*={w.temperature}, "
                        f"rc=2.5 sigma force-shifted, dt={w.dt}, NVE, cell list rebuilt every step, "
                        f"FP64 U/K/W every {thermo_every} steps",
            "n": w.n,
            "box": box,
            "cells_per_dim": s.cells_per_dim,
            "thermo_every": thermo_every,
        },
        "roofline": {
            "kernel": "k_forces<false,false,true,false,1> (md_forces)",
            "state": f"after the {args.warmup} warm-up steps",
            **roof,
            "traffic": recorded_traffic(args.workload),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
        },
        "thermo_last": e_th,
        "timed_region": {"hip_events_ms": gpu_s * 1e3, "wall_ms": wall * 1e3},
    }
    if args.copy_calibration_mib > 0:
        # one plain copy of known size: FETCH_SIZE/WRITE_SIZE of this dispatch give the
        # counter-to-bytes factor for the traffic figures
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nbytes
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(torch)
        out["adjoint"]["ratio_vs_plain_headline"] = out["adjoint"]["value"] / value
    if not args.no_batched:
        out["batched"] = batched_leg(torch)
        out["batched"]["ratio_vs_plain_headline"] = out["batched"]["value"] / value
    if not args.no_widened:
        out["full_size"] = full_size_leg(torch)
        out["density_axis"] = density_leg(torch)
        out["wca"] = wca_leg(torch)
        out["skin"] = skin_leg(torch)
        out["pair_list"] = pair_list_leg(torch)
        out["neighbor_list"] = pair_list_leg(torch, atom_lists=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s.state()[0].cpu().numpy(), box, args.cpu_seconds)
        sp, sv = s.state()
        out["cpu_cell_list"] = cpu_cell_list(sp.cpu().numpy(), sv.cpu().numpy(), box, value)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
