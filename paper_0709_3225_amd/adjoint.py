"""Differentiating an LJ velocity-Verlet trajectory through the HIP library.

`LJTrajectory` is a torch.autograd.Function: its forward advances a state T
steps with md_step and returns the library's md_loss, L = K_T / N +
W_T / (3 V) (mean kinetic energy per particle plus the virial part of the
pressure, FP64); its backward seeds the adjoint with md_adjoint_seed and runs
the discrete adjoint of velocity Verlet segment by segment, last segment
first. Each segment of `every` steps is recomputed from a checkpoint
(positions and velocities saved every `every` steps in the forward) with
md_adjoint_recompute on a second stream and workspace, one segment ahead of
the sweep (md_adjoint_path) that runs the adjoints of the segment before it,
so the two overlap on the GPU; two path buffers alternate between them. With
keep_path the forward keeps every state instead (md_step_path, 16 N + 4 n_c^3
bytes per step) and the backward only sweeps. Every variant gives bitwise the
same gradients as md_adjoint_segment called segment by segment.

With h = dt / (2 m), one Verlet step is v' = v + h F(r), r' = r + dt v',
v'' = v' + h F(r'). Its transpose, applied from the last step back, is a kick
adjoint at r' (lam_r += h J(r') lam_v, J = dF/dr), a drift adjoint
(lam_v += dt lam_r) and a kick adjoint at r with the new lam_v. The kick
adjoint at r_n of step n and the one of step n - 1 use the same vector, so
interior positions get one kick adjoint with coefficient 2 h.

Only argument marshalling happens here: every vector operation runs in the
library's kernels.
"""
from __future__ import annotations

import torch

from . import _lib as L


class _Runner:
    """Workspace and parameters of one trajectory."""

    def __init__(self, n, box, eps, sigma, mass, dt, device):
        self.n = int(n)
        self.box = float(box)
        self.p = L.make_params(n, box, float(eps), float(sigma), mass, 2.5, dt)
        self.dev = device
        self.ws = torch.empty(L.md_workspace_bytes(self.p), dtype=torch.uint8, device=device)

    def vec(self):
        return torch.zeros((self.n, 4), dtype=torch.float32, device=self.dev)


def _segments(nsteps, every):
    return [(n0, min(every, nsteps - n0)) for n0 in range(0, nsteps, every)]


def _forward(run: _Runner, pos4, vel4, nsteps, every, keep_path=False):
    """Loss, checkpoints [(first step, steps, pos4, vel4)] and the kept path
    (path4, path_start) or None."""
    L.md_build_cells(run.p, run.ws, pos4, vel4)
    L.md_forces(run.p, run.ws)
    ckpts, kept = [], None
    if keep_path:
        nc, _ = L.md_cell_grid(run.p)
        path = torch.empty((nsteps, run.n, 4), dtype=torch.float32, device=run.dev)
        path_start = torch.empty((nsteps, nc ** 3 + 1), dtype=torch.int32, device=run.dev)
        L.md_step_path(run.p, run.ws, nsteps, path, path_start)
        kept = (path, path_start)
        ckpts = [(n0, k, None, None) for n0, k in _segments(nsteps, every)]
    else:
        for n0, k in _segments(nsteps, every):
            cp, cv = run.vec(), run.vec()
            L.md_get_state(run.p, run.ws, cp, cv)
            ckpts.append((n0, k, cp, cv))
            L.md_step(run.p, run.ws, k)
    loss = torch.empty(1, dtype=torch.float64, device=run.dev)
    L.md_loss(run.p, run.ws, loss)
    return loss[0], ckpts, kept


def _backward(run: _Runner, ckpts, gl: float, every, kept=None, overlap=True):
    lam_r, lam_v = run.vec(), run.vec()
    theta = torch.zeros(2, dtype=torch.float64, device=run.dev)
    # the workspace still holds the final state r_T, v_T
    L.md_adjoint_seed(run.p, run.ws, gl, lam_r, lam_v, theta)
    segs = list(reversed(ckpts))
    if kept is not None:
        path, path_start = kept
        for n0, k, _, _ in segs:
            L.md_adjoint_path(run.p, run.ws, n0, k, path[n0:n0 + k], path_start[n0:n0 + k], lam_r, lam_v, theta)
        L.md_check(run.ws)
        return lam_r, lam_v, theta
    nc, _ = L.md_cell_grid(run.p)
    bufs = [(torch.empty((every, run.n, 4), dtype=torch.float32, device=run.dev),
             torch.empty((every, nc ** 3 + 1), dtype=torch.int32, device=run.dev)) for _ in range(2 if overlap else 1)]
    if not overlap:
        path, path_start = bufs[0]
        for n0, k, cp, cv in segs:
            # recompute r_{n0} .. r_{n0+k-1}, then the drift and kick adjoints
            # of steps n0+k-1 .. n0 (one library call per segment)
            L.md_adjoint_segment(run.p, run.ws, cp, cv, n0, k, path, path_start, lam_r, lam_v, theta)
        L.md_check(run.ws)
        return lam_r, lam_v, theta
    main = torch.cuda.current_stream(run.dev)
    side = torch.cuda.Stream(device=run.dev)  # default priority
    ws2 = torch.empty_like(run.ws)
    freed = [None, None]  # per buffer: the sweep that read it last

    def recompute(i):
        # segment i (last segment first) into buffer i % 2, once the sweep
        # that read that buffer before has finished
        _, k, cp, cv = segs[i]
        path, path_start = bufs[i % 2]
        if freed[i % 2] is not None:
            side.wait_event(freed[i % 2])
        L.md_adjoint_recompute(run.p, ws2, cp, cv, k, path, path_start, stream=side)
        done = torch.cuda.Event()
        done.record(side)
        return done

    side.wait_stream(main)  # checkpoints, seed and buffers are ready
    ready = recompute(0)
    for i, (n0, k, _, _) in enumerate(segs):
        nxt = recompute(i + 1) if i + 1 < len(segs) else None
        main.wait_event(ready)
        path, path_start = bufs[i % 2]
        L.md_adjoint_path(run.p, run.ws, n0, k, path, path_start, lam_r, lam_v, theta, stream=main)
        freed[i % 2] = torch.cuda.Event()
        freed[i % 2].record(main)
        ready = nxt
    # every recompute has been waited for by a sweep on the main stream
    L.md_check(run.ws)
    L.md_check(ws2)
    return lam_r, lam_v, theta


def trajectory_gradients(pos4, vel4, box, eps=1.0, sigma=1.0, mass=1.0, dt=0.005, nsteps=200, every=20,
                         keep_path=False, overlap=True):
    """(L, dL/dr0 [N,4], dL/dv0 [N,4], dL/deps, dL/dsigma) for L = K_T/N + W_T/(3V).

    keep_path: keep every state in the forward (no recomputation); overlap:
    recompute the next segment on a second stream while the current one is
    swept (False: one md_adjoint_segment call per segment, on one stream)."""
    run = _Runner(pos4.shape[0], box, eps, sigma, mass, dt, pos4.device)
    loss, ckpts, kept = _forward(run, pos4.contiguous(), vel4.contiguous(), nsteps, every, keep_path)
    gr, gv, th = _backward(run, ckpts, 1.0, every, kept, overlap)
    th = th.cpu()
    return float(loss), gr, gv, float(th[0]), float(th[1])


class LJTrajectory(torch.autograd.Function):
    """loss = LJTrajectory.apply(pos4, vel4, eps, sigma, box, mass, dt, nsteps, every, keep_path)."""

    @staticmethod
    def forward(ctx, pos4, vel4, eps, sigma, box, mass=1.0, dt=0.005, nsteps=200, every=20, keep_path=False):
        run = _Runner(pos4.shape[0], box, float(eps), float(sigma), mass, dt, pos4.device)
        loss, ckpts, kept = _forward(run, pos4.detach().contiguous(), vel4.detach().contiguous(), int(nsteps),
                                     int(every), bool(keep_path))
        ctx.run, ctx.ckpts, ctx.every, ctx.kept = run, ckpts, int(every), kept
        ctx.eps_like, ctx.sig_like = eps, sigma
        return loss

    @staticmethod
    def backward(ctx, grad_out):
        gr, gv, th = _backward(ctx.run, ctx.ckpts, float(grad_out), ctx.every, ctx.kept)
        ge = th[0].to(ctx.eps_like.dtype).to(ctx.eps_like.device) if torch.is_tensor(ctx.eps_like) else None
        gs = th[1].to(ctx.sig_like.dtype).to(ctx.sig_like.device) if torch.is_tensor(ctx.sig_like) else None
        return gr, gv, ge, gs, None, None, None, None, None, None
