"""Pins for the oracle's derivative functions and the reference trajectory
gradient (CPU only).

The Hessian-vector product, the parameter derivatives of the force sum and the
virial gradient are fixed by central finite differences of the pinned force
and virial sums, by the symmetry of the Hessian, by the translation null space
and by the linearity in epsilon. The torch reference gradient is fixed by an
independent forward (the C oracle's velocity Verlet) and by central finite
differences of that forward.
"""
import numpy as np
import pytest

import ljsynth


def _state(amp=0.1, name="lj256_check"):
    w = ljsynth.WORKLOADS[name]
    pos4, vel4, box = ljsynth.make_state(w, jitter_amp=amp)
    return pos4[:, :3].astype(np.float64), vel4[:, :3].astype(np.float64), box


def test_hvp_matches_force_differences(orc):
    pos, _, box = _state()
    p = orc.params(box)
    u = np.random.default_rng(1).normal(size=pos.shape)
    ju = orc.hvp(p, pos, u)
    h = 1e-6
    fp, _, _ = orc.forces(p, pos + h * u)
    fm, _, _ = orc.forces(p, pos - h * u)
    fd = (fp - fm) / (2 * h)
    assert np.linalg.norm(ju - fd) <= 1e-6 * np.linalg.norm(fd)


def test_hvp_symmetric_and_translation_free(orc):
    pos, _, box = _state()
    p = orc.params(box)
    rng = np.random.default_rng(2)
    u, w = rng.normal(size=pos.shape), rng.normal(size=pos.shape)
    a = float((u * orc.hvp(p, pos, w)).sum())
    b = float((w * orc.hvp(p, pos, u)).sum())
    assert a == pytest.approx(b, rel=1e-12)
    t = np.zeros_like(pos)
    t[:, 0] = 1.0
    assert np.abs(orc.hvp(p, pos, t)).max() < 1e-11


def test_hvp_two_atoms_closed_form(orc):
    """Two atoms on the x axis at distance r: moving atom 0 by u along x changes
    its force by phi'(r) u (the Jacobian block is phi' along the bond and phi/r
    across it)."""
    p = orc.params(10.0)
    r = 1.1
    pos = np.array([[2.0, 5.0, 5.0], [2.0 + r, 5.0, 5.0]])
    h = 1e-6
    phi_p, _ = orc.pair(p, r + h)
    phi_m, _ = orc.pair(p, r - h)
    dphi = (phi_p - phi_m) / (2 * h)
    phi, _ = orc.pair(p, r)
    ux = orc.hvp(p, pos, np.array([[1.0, 0, 0], [0, 0, 0]]))
    uy = orc.hvp(p, pos, np.array([[0.0, 1.0, 0], [0, 0, 0]]))
    # F_0x = -phi(x1 - x0), so dF_0x/dx0 = phi'(r) and dF_1x/dx0 = -phi'(r)
    assert ux[0, 0] == pytest.approx(dphi, rel=1e-7)
    assert ux[1, 0] == pytest.approx(-dphi, rel=1e-7)
    assert uy[0, 1] == pytest.approx(phi / r, rel=1e-10)


def test_force_parameter_derivatives(orc):
    pos, _, box = _state()
    a = np.random.default_rng(3).normal(size=pos.shape)
    de, ds = orc.dforce_dparams(orc.params(box), pos, a)
    h = 1e-6
    fe = [(a * orc.forces(orc.params(box, epsilon=1 + s * h), pos)[0]).sum() for s in (1, -1)]
    fs = [(a * orc.forces(orc.params(box, sigma=1 + s * h), pos)[0]).sum() for s in (1, -1)]
    assert de == pytest.approx((fe[0] - fe[1]) / (2 * h), rel=1e-7)
    assert ds == pytest.approx((fs[0] - fs[1]) / (2 * h), rel=1e-6)
    # linear in epsilon
    f, _, _ = orc.forces(orc.params(box), pos)
    assert de == pytest.approx((a * f).sum(), rel=1e-12)


def test_virial_gradient(orc):
    pos, _, box = _state()
    p = orc.params(box)
    g, dwe, dws = orc.virial_grad(p, pos)
    _, _, W = orc.forces(p, pos)
    rng = np.random.default_rng(4)
    u = rng.normal(size=pos.shape)
    h = 1e-6
    wp = orc.forces(p, pos + h * u)[2]
    wm = orc.forces(p, pos - h * u)[2]
    assert (g * u).sum() == pytest.approx((wp - wm) / (2 * h), rel=1e-6)
    assert dwe == pytest.approx(W, rel=1e-12)  # W is linear in epsilon
    ws = [orc.forces(orc.params(box, sigma=1 + s * h), pos)[2] for s in (1, -1)]
    assert dws == pytest.approx((ws[0] - ws[1]) / (2 * h), rel=1e-6)


def test_energy_shift_mode_refused(orc):
    pos, _, box = _state()
    with pytest.raises(ValueError):
        orc.hvp(orc.params(box, shift_mode=1), pos, pos)


# ------------------------------------------------------- trajectory gradient

NSTEPS = 200


@pytest.fixture(scope="module")
def traj():
    pos, vel, box = _state(amp=0.05)
    return pos, vel, box


def _c_loss(orc, pos, vel, box, eps=1.0, sigma=1.0, nsteps=NSTEPS):
    p = orc.params(box, epsilon=eps, sigma=sigma)
    x, v, th = orc.run(p, pos, vel, nsteps)
    return th[-1, 1] / len(pos) + th[-1, 2] / (3 * box ** 3)


def test_reference_forward_matches_c_oracle(orc, traj):
    from oracle import grad_ref

    pos, vel, box = traj
    loss, *_ = grad_ref.loss_and_grads(pos, vel, box, nsteps=NSTEPS)
    assert loss == pytest.approx(_c_loss(orc, pos, vel, box), rel=1e-10)


def test_reference_gradient_matches_finite_differences(orc, traj):
    from oracle import grad_ref

    pos, vel, box = traj
    loss, gx, gv, ge, gs = grad_ref.loss_and_grads(pos, vel, box, nsteps=NSTEPS)
    h = 1e-6
    le = [_c_loss(orc, pos, vel, box, eps=1 + s * h) for s in (1, -1)]
    ls = [_c_loss(orc, pos, vel, box, sigma=1 + s * h) for s in (1, -1)]
    assert ge == pytest.approx((le[0] - le[1]) / (2 * h), rel=1e-5)
    assert gs == pytest.approx((ls[0] - ls[1]) / (2 * h), rel=1e-5)
    rng = np.random.default_rng(5)
    for _ in range(3):
        i, c = int(rng.integers(len(pos))), int(rng.integers(3))
        for g, arr, which in ((gx, pos, "x"), (gv, vel, "v")):
            pp = arr.copy()
            pp[i, c] += h
            lp = _c_loss(orc, pp, vel, box) if which == "x" else _c_loss(orc, pos, pp, box)
            pp[i, c] -= 2 * h
            lm = _c_loss(orc, pp, vel, box) if which == "x" else _c_loss(orc, pos, pp, box)
            assert g[i, c] == pytest.approx((lp - lm) / (2 * h), rel=1e-4, abs=1e-7)
