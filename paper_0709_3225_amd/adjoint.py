"""Differentiating an LJ velocity-Verlet trajectory through the HIP library.

`LJTrajectory` is a torch.autograd.Function: its forward advances a state T
steps with md_step and returns the library's md_loss, L = K_T / N +
W_T / (3 V) (mean kinetic energy per particle plus the virial part of the
pressure, FP64); its backward seeds the adjoint with md_adjoint_seed and runs
the discrete adjoint of velocity Verlet with md_adjoint_segment, recomputing
each segment of `every` steps from a checkpoint (positions and velocities
saved every `every` steps in the forward).

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


def _forward(run: _Runner, pos4, vel4, nsteps, every):
    L.md_build_cells(run.p, run.ws, pos4, vel4)
    L.md_forces(run.p, run.ws)
    ckpts = []
    done = 0
    while done < nsteps:
        k = min(every, nsteps - done)
        cp, cv = run.vec(), run.vec()
        L.md_get_state(run.p, run.ws, cp, cv)
        ckpts.append((done, k, cp, cv))
        L.md_step(run.p, run.ws, k)
        done += k
    loss = torch.empty(1, dtype=torch.float64, device=run.dev)
    L.md_loss(run.p, run.ws, loss)
    return loss[0], ckpts


def _backward(run: _Runner, ckpts, gl: float, every):
    lam_r, lam_v = run.vec(), run.vec()
    theta = torch.zeros(2, dtype=torch.float64, device=run.dev)
    # the workspace still holds the final state r_T, v_T
    L.md_adjoint_seed(run.p, run.ws, gl, lam_r, lam_v, theta)
    path = torch.empty((every, run.n, 4), dtype=torch.float32, device=run.dev)
    nc, _ = L.md_cell_grid(run.p)
    path_start = torch.empty((every, nc ** 3 + 1), dtype=torch.int32, device=run.dev)
    for n0, k, cp, cv in reversed(ckpts):
        # recompute r_{n0} .. r_{n0+k-1}, then the drift and kick adjoints of
        # steps n0+k-1 .. n0 (one library call per segment)
        L.md_adjoint_segment(run.p, run.ws, cp, cv, n0, k, path, path_start, lam_r, lam_v, theta)
    L.md_check(run.ws)
    return lam_r, lam_v, theta


def trajectory_gradients(pos4, vel4, box, eps=1.0, sigma=1.0, mass=1.0, dt=0.005, nsteps=200, every=20):
    """(L, dL/dr0 [N,4], dL/dv0 [N,4], dL/deps, dL/dsigma) for L = K_T/N + W_T/(3V)."""
    run = _Runner(pos4.shape[0], box, eps, sigma, mass, dt, pos4.device)
    loss, ckpts = _forward(run, pos4.contiguous(), vel4.contiguous(), nsteps, every)
    gr, gv, th = _backward(run, ckpts, 1.0, every)
    th = th.cpu()
    return float(loss), gr, gv, float(th[0]), float(th[1])


class LJTrajectory(torch.autograd.Function):
    """loss = LJTrajectory.apply(pos4, vel4, eps, sigma, box, mass, dt, nsteps, every)."""

    @staticmethod
    def forward(ctx, pos4, vel4, eps, sigma, box, mass=1.0, dt=0.005, nsteps=200, every=20):
        run = _Runner(pos4.shape[0], box, float(eps), float(sigma), mass, dt, pos4.device)
        loss, ckpts = _forward(run, pos4.detach().contiguous(), vel4.detach().contiguous(), int(nsteps), int(every))
        ctx.run, ctx.ckpts, ctx.every = run, ckpts, int(every)
        ctx.eps_like, ctx.sig_like = eps, sigma
        return loss

    @staticmethod
    def backward(ctx, grad_out):
        gr, gv, th = _backward(ctx.run, ctx.ckpts, float(grad_out), ctx.every)
        ge = th[0].to(ctx.eps_like.dtype).to(ctx.eps_like.device) if torch.is_tensor(ctx.eps_like) else None
        gs = th[1].to(ctx.sig_like.dtype).to(ctx.sig_like.device) if torch.is_tensor(ctx.sig_like) else None
        return gr, gv, ge, gs, None, None, None, None, None
