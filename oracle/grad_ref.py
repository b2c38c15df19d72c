"""Reference gradient of a velocity-Verlet LJ trajectory (test infrastructure).

A second, independent FP64 implementation of the same dynamics as the C
oracle, written with plain PyTorch CPU tensor operations so that autograd can
differentiate it: the all-pairs force sum of section 2 (truncated at
r_c = 2.5 sigma, force shifted to zero at the cutoff), minimum image in a
cubic periodic box, and velocity Verlet (kick, drift, wrap, force, kick).

The loss is the mean kinetic energy per particle plus the virial part of the
pressure at the final step, L = K_T / N + W_T / (3 V), with W the sum over
pairs of r phi(r). Gradients are taken with respect to the initial positions,
the initial velocities, epsilon and sigma (r_c moves with sigma).

Only tests import this module; it shares nothing with the GPU library.
"""
from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint


def _flj(r, eps, sigma):
    """LJ pair force magnitude -du_LJ/dr = (24 eps / r) [2 (sigma/r)^12 - (sigma/r)^6]."""
    sr6 = (sigma / r) ** 6
    return 24.0 * eps / r * (2.0 * sr6 * sr6 - sr6)


def forces_and_virial(x, box, eps, sigma, rc_over_sigma=2.5):
    """All-pairs truncated, force-shifted LJ forces [N,3] and virial W."""
    n = x.shape[0]
    rc = rc_over_sigma * sigma
    d = x[:, None, :] - x[None, :, :]
    d = d - box * torch.round(d / box)  # round half to even, like rint
    r2 = (d * d).sum(-1)
    off = ~torch.eye(n, dtype=torch.bool)
    inside = off & (r2 < rc * rc)
    r = torch.sqrt(torch.where(inside, r2, torch.ones_like(r2)))
    phi = torch.where(inside, _flj(r, eps, sigma) - _flj(rc, eps, sigma), torch.zeros_like(r2))
    f = ((phi / r)[..., None] * d).sum(1)
    w = 0.5 * (r * phi).sum()
    return f, w


def _wrap(x, box):
    return x - box * torch.floor(x / box)


def _segment(x, v, f, eps, sigma, box, mass, dt, nsteps):
    h = 0.5 * dt / mass
    for _ in range(nsteps):
        v = v + h * f
        x = _wrap(x + dt * v, box)
        f, _ = forces_and_virial(x, box, eps, sigma)
        v = v + h * f
    return x, v, f


def trajectory_loss(x0, v0, eps, sigma, box, mass, dt, nsteps, segment=20):
    """L = K_T/N + W_T/(3V) after nsteps velocity-Verlet steps (FP64 tensors).

    Segments of `segment` steps are checkpointed so memory stays bounded.
    """
    n = x0.shape[0]
    f, _ = forces_and_virial(x0, box, eps, sigma)
    x, v = x0, v0
    done = 0
    while done < nsteps:
        k = min(segment, nsteps - done)
        x, v, f = checkpoint(_segment, x, v, f, eps, sigma, box, mass, dt, k, use_reentrant=False)
        done += k
    _, w = forces_and_virial(x, box, eps, sigma)
    kin = 0.5 * mass * (v * v).sum()
    return kin / n + w / (3.0 * box ** 3)


def loss_and_grads(pos, vel, box, eps=1.0, sigma=1.0, mass=1.0, dt=0.005, nsteps=200):
    """Loss value and (dL/dr0 [N,3], dL/dv0 [N,3], dL/deps, dL/dsigma), all FP64."""
    x0 = torch.tensor(pos[:, :3], dtype=torch.float64, requires_grad=True)
    v0 = torch.tensor(vel[:, :3], dtype=torch.float64, requires_grad=True)
    e = torch.tensor(float(eps), dtype=torch.float64, requires_grad=True)
    s = torch.tensor(float(sigma), dtype=torch.float64, requires_grad=True)
    loss = trajectory_loss(x0, v0, e, s, float(box), float(mass), float(dt), int(nsteps))
    gx, gv, ge, gs = torch.autograd.grad(loss, (x0, v0, e, s))
    return float(loss.detach()), gx.numpy(), gv.numpy(), float(ge), float(gs)
