"""GPU parity of the adjoint entry points against the FP64 oracle.

Single-state kernels (Hessian-vector product, force parameter derivatives,
virial gradient) are compared with the oracle's pinned FP64 functions at
1e-5 relative. The trajectory gradient of L = K_T/N + W_T/(3V) through 200
velocity-Verlet steps (N = 256, checkpoints every 20 steps) is compared with
the torch-float64 reference: FP32 and FP64 trajectories separate
exponentially over one time unit, so the bound is 1e-3 relative L2 for the
position and velocity gradients and 1e-4 relative for d/d(eps, sigma).
"""
import numpy as np
import pytest

import ljsynth

pytestmark = pytest.mark.gpu

REL = 1e-5


def _torch():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _dev(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _loaded(pos4, box, vel4=None, waves=0, tile=0):
    from paper_0709_3225_amd import LJSystem

    s = LJSystem(len(pos4), box, waves_per_cell=waves, tile_cap=tile)
    s.load(_dev(pos4), None if vel4 is None else _dev(vel4), forces=False)
    return s


# dense grids of 8 to 2,197 cells, and a sparse one of 19,683 cells
HVP_CASES = {
    "lj256_check": lambda: ljsynth.WORKLOADS["lj256_check"],
    "lj4k": lambda: ljsynth.WORKLOADS["lj4k"],
    "lj32k_adjoint": lambda: ljsynth.WORKLOADS["lj32k_adjoint"],
    "rho0.1_32k": lambda: ljsynth.Workload("rho0.1_32k", 20, 0.1, 1.0, 0, 55),
}


@pytest.mark.parametrize("waves", [1, 2, 4])
@pytest.mark.parametrize("name", list(HVP_CASES))
def test_hvp_and_force_parameter_derivatives(name, waves, orc):
    """The pair pass with one, two or four wavefronts per cell (each
    wavefront screens and walks its own range of the candidates)."""
    torch = _torch()
    from paper_0709_3225_amd import _lib as L

    pos4, vel4, box = ljsynth.make_state(HVP_CASES[name](), jitter_amp=0.05, shuffle=True)
    _say(f"hvp {name} n={len(pos4)} waves={waves}")
    w = np.zeros_like(pos4)
    w[:, :3] = np.random.default_rng(7).normal(size=(len(pos4), 3))
    s = _loaded(pos4, box, waves=waves)
    lam = torch.zeros((len(pos4), 4), dtype=torch.float32, device="cuda")
    theta = torch.zeros(2, dtype=torch.float64, device="cuda")
    L.md_adjoint_kick(s.params, s.ws, _dev(w), lam, theta, 1.0)
    assert s.check() == 0
    ju = lam.cpu().numpy()[:, :3].astype(np.float64)
    p = orc.params(box)
    ref = orc.hvp(p, pos4, w)
    assert rel_l2(ju, ref) <= REL
    # accumulation: a second call with coef -0.5 halves lam
    L.md_adjoint_kick(s.params, s.ws, _dev(w), lam, None, -0.5)
    assert rel_l2(lam.cpu().numpy()[:, :3], 0.5 * ref) <= REL
    # parameter derivatives projected on the forces themselves (w = F): the sums
    # sum_i F_i . dF_i/d(eps, sigma) do not cancel, so 1e-5 relative is meaningful
    # (a random w makes them cancel by orders of magnitude)
    f, _, _ = orc.forces(p, pos4)
    wf = np.zeros_like(pos4)
    wf[:, :3] = f
    theta.zero_()
    L.md_adjoint_kick(s.params, s.ws, _dev(wf), lam, theta, 1.0)
    assert s.check() == 0
    de, ds = orc.dforce_dparams(p, pos4, f)
    th = theta.cpu().numpy()
    assert th[0] == pytest.approx(de, rel=REL)
    assert th[1] == pytest.approx(ds, rel=REL)


@pytest.mark.parametrize("k", [1, 4, 8, 10, 12, 16, 17, 20, 24])
def test_hvp_every_home_layout(k, orc):
    """The pair pass on every home-cell lane layout on its own (exactly k
    atoms in every cell: the VALU screen with 16 down to 6 slices, the
    matrix-core screen, three and two slices): Hessian-vector product and
    virial gradient against the oracle."""
    torch = _torch()
    from paper_0709_3225_amd import _lib as L

    pos4, box = ljsynth.k_per_cell(k, 200 + k)
    _say(f"hvp home layout k={k} n={len(pos4)}")
    w = np.zeros_like(pos4)
    w[:, :3] = np.random.default_rng(k).normal(size=(len(pos4), 3))
    p = orc.params(box)
    s = _loaded(pos4, box)
    assert s.cells_per_dim == 4
    lam = torch.zeros((len(pos4), 4), dtype=torch.float32, device="cuda")
    L.md_adjoint_kick(s.params, s.ws, _dev(w), lam, None, 1.0)
    assert s.check() == 0
    assert rel_l2(lam.cpu().numpy()[:, :3].astype(np.float64), orc.hvp(p, pos4, w)) <= REL
    gref, _, _ = orc.virial_grad(p, pos4)
    gr = torch.zeros((len(pos4), 4), dtype=torch.float32, device="cuda")
    gv = torch.zeros((len(pos4), 4), dtype=torch.float32, device="cuda")
    L.md_loss_grad(s.params, s.ws, 0.0, 1.0, gr, gv, None)
    assert s.check() == 0
    assert rel_l2(gr.cpu().numpy()[:, :3].astype(np.float64), gref) <= REL


@pytest.mark.parametrize("tile", [192, 1024])
@pytest.mark.parametrize("name", ["lj4k", "lj32k_adjoint"])
def test_hvp_with_lds_tile(name, tile, orc):
    """The pair pass with a 192-atom LDS tile (every neighbourhood in several
    passes, staged through the segment table, with the adjoint vector's tile
    beside it) and with a 1,024-atom one: Hessian-vector product and loss
    gradient against the oracle, in one and four wavefronts per cell."""
    torch = _torch()
    from paper_0709_3225_amd import _lib as L

    pos4, vel4, box = ljsynth.make_state(HVP_CASES[name](), jitter_amp=0.05, shuffle=True)
    _say(f"hvp {name} n={len(pos4)} tile={tile}")
    w = np.zeros_like(pos4)
    w[:, :3] = np.random.default_rng(9).normal(size=(len(pos4), 3))
    p = orc.params(box)
    ref = orc.hvp(p, pos4, w)
    gref, _, _ = orc.virial_grad(p, pos4)
    for waves in (1, 4):
        s = _loaded(pos4, box, waves=waves, tile=tile)
        assert L.md_tile_capacity(s.params) == tile
        lam = torch.zeros((len(pos4), 4), dtype=torch.float32, device="cuda")
        L.md_adjoint_kick(s.params, s.ws, _dev(w), lam, None, 1.0)
        assert s.check() == 0
        assert rel_l2(lam.cpu().numpy()[:, :3].astype(np.float64), ref) <= REL
        gr = torch.zeros((len(pos4), 4), dtype=torch.float32, device="cuda")
        gv = torch.zeros((len(pos4), 4), dtype=torch.float32, device="cuda")
        L.md_loss_grad(s.params, s.ws, 0.0, 1.0, gr, gv, None)
        assert s.check() == 0
        assert rel_l2(gr.cpu().numpy()[:, :3].astype(np.float64), gref) <= REL


def test_hvp_symmetry_and_translation():
    torch = _torch()
    from paper_0709_3225_amd import _lib as L

    pos4, vel4, box = ljsynth.make_state(ljsynth.WORKLOADS["lj4k"], jitter_amp=0.05)
    _say("hvp symmetry lj4k")
    s = _loaded(pos4, box)
    rng = np.random.default_rng(8)
    u = np.zeros_like(pos4)
    v = np.zeros_like(pos4)
    u[:, :3] = rng.normal(size=(len(pos4), 3))
    v[:, :3] = rng.normal(size=(len(pos4), 3))
    outs = []
    for a_ in (u, v):
        lam = torch.zeros((len(pos4), 4), dtype=torch.float32, device="cuda")
        L.md_adjoint_kick(s.params, s.ws, _dev(a_), lam, None, 1.0)
        outs.append(lam.cpu().numpy().astype(np.float64))
    a = float((u * outs[1]).sum())
    b = float((v * outs[0]).sum())
    assert a == pytest.approx(b, rel=1e-4)
    t = np.zeros_like(pos4)
    t[:, 1] = 1.0
    lam = torch.zeros((len(pos4), 4), dtype=torch.float32, device="cuda")
    L.md_adjoint_kick(s.params, s.ws, _dev(t), lam, None, 1.0)
    assert np.abs(lam.cpu().numpy()).max() <= 1e-6 * np.abs(outs[0]).max()
    assert s.check() == 0


@pytest.mark.parametrize("waves", [1, 4])
@pytest.mark.parametrize("name", ["lj256_check", "lj4k", "rho0.1_32k"])
def test_loss_gradient(name, waves, orc):
    torch = _torch()
    from paper_0709_3225_amd import _lib as L

    pos4, vel4, box = ljsynth.make_state(HVP_CASES[name](), jitter_amp=0.05)
    _say(f"loss gradient {name} waves={waves}")
    n = len(pos4)
    s = _loaded(pos4, box, vel4, waves=waves)
    gr = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    gv = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    theta = torch.zeros(2, dtype=torch.float64, device="cuda")
    kc, wc = 1.0 / n, 1.0 / (3 * box ** 3)
    L.md_loss_grad(s.params, s.ws, kc, wc, gr, gv, theta)
    assert s.check() == 0
    g, dwe, dws = orc.virial_grad(orc.params(box), pos4)
    assert rel_l2(gr.cpu().numpy()[:, :3], wc * g) <= REL
    np.testing.assert_allclose(gv.cpu().numpy()[:, :3], kc * vel4[:, :3], rtol=1e-6)
    th = theta.cpu().numpy()
    assert th[0] == pytest.approx(wc * dwe, rel=REL)
    assert th[1] == pytest.approx(wc * dws, rel=REL)


def test_adjoint_drift():
    torch = _torch()
    from paper_0709_3225_amd import _lib as L, make_params

    _say("adjoint drift")
    n = 1000
    p = make_params(n, 10.0, dt=0.005)
    a = torch.randn((n, 4), device="cuda")
    b = torch.randn((n, 4), device="cuda")
    ref = b.clone()
    ref[:, :3] += 0.005 * a[:, :3]
    L.md_adjoint_drift(p, a, b)
    torch.cuda.synchronize()
    assert torch.allclose(b[:, :3], ref[:, :3], rtol=1e-6, atol=1e-7)


def test_energy_shift_mode_refused():
    torch = _torch()
    from paper_0709_3225_amd import _lib as L, LJSystem, MDError

    _say("adjoint refuses shift_mode 1")
    pos4, vel4, box = ljsynth.make_state(ljsynth.WORKLOADS["lj256_check"])
    s = LJSystem(len(pos4), box, shift_mode=1)
    s.load(_dev(pos4), forces=False)
    lam = torch.zeros((len(pos4), 4), dtype=torch.float32, device="cuda")
    with pytest.raises(MDError):
        L.md_adjoint_kick(s.params, s.ws, _dev(pos4), lam, None, 1.0)


def test_trajectory_gradient_matches_fp64_reference():
    torch = _torch()
    from oracle import grad_ref
    from paper_0709_3225_amd import trajectory_gradients

    w = ljsynth.WORKLOADS["lj256_check"]
    pos4, vel4, box = ljsynth.make_state(w, jitter_amp=0.05)
    _say("trajectory gradient n=256 T=200 every=20")
    loss, gr, gv, ge, gs = trajectory_gradients(_dev(pos4), _dev(vel4), box, nsteps=200, every=20)
    rl, rx, rv, re, rs = grad_ref.loss_and_grads(pos4, vel4, box, nsteps=200)
    assert loss == pytest.approx(rl, rel=1e-4)
    assert rel_l2(gr.cpu().numpy()[:, :3], rx) <= 1e-3
    assert rel_l2(gv.cpu().numpy()[:, :3], rv) <= 1e-3
    assert ge == pytest.approx(re, rel=1e-4)
    assert gs == pytest.approx(rs, rel=1e-4)


def test_autograd_function_matches_direct_call():
    torch = _torch()
    from paper_0709_3225_amd import LJTrajectory, trajectory_gradients

    w = ljsynth.WORKLOADS["lj256_check"]
    pos4, vel4, box = ljsynth.make_state(w, jitter_amp=0.05)
    _say("autograd function n=256 T=40")
    x = _dev(pos4).requires_grad_(True)
    v = _dev(vel4).requires_grad_(True)
    e = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    sg = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    loss = LJTrajectory.apply(x, v, e, sg, box, 1.0, 0.005, 40, 10)
    loss.backward()
    l2, gr, gv, ge, gs = trajectory_gradients(_dev(pos4), _dev(vel4), box, nsteps=40, every=10)
    assert float(loss) == l2
    assert torch.equal(x.grad, gr) and torch.equal(v.grad, gv)
    assert float(e.grad) == ge and float(sg.grad) == gs


@pytest.mark.parametrize("wl,nsteps,every", [("lj4k", 45, 10), ("lj32k_adjoint", 40, 20)])
def test_backward_modes_bitwise_equal(wl, nsteps, every):
    """Three ways to run the backward pass give bitwise the same loss and
    gradients: one md_adjoint_segment call per segment on one stream; the
    overlapped form (md_adjoint_recompute of the next segment on a second
    stream and workspace while md_adjoint_path sweeps the current one, two
    path buffers alternating); and the kept path (md_step_path in the
    forward, md_adjoint_path over slices of it, no recomputation). A short
    last segment is included (45 = 4 x 10 + 5)."""
    torch = _torch()
    from paper_0709_3225_amd import trajectory_gradients

    w = ljsynth.WORKLOADS[wl]
    pos4, vel4, box = ljsynth.make_state(w, jitter_amp=0.05)
    x, v = _dev(pos4), _dev(vel4)
    out = {}
    for mode, kw in (("segment", dict(overlap=False)), ("overlap", dict(overlap=True)),
                     ("kept", dict(keep_path=True))):
        _say(f"backward mode {mode} n={len(pos4)} T={nsteps} every={every}")
        out[mode] = trajectory_gradients(x, v, box, dt=w.dt, nsteps=nsteps, every=every, **kw)
        torch.cuda.synchronize()
    ref = out["segment"]
    assert np.isfinite(ref[0]) and float(ref[1].abs().sum()) > 0.0
    for mode in ("overlap", "kept"):
        got = out[mode]
        assert got[0] == ref[0], mode
        assert torch.equal(got[1], ref[1]) and torch.equal(got[2], ref[2]), mode
        assert got[3] == ref[3] and got[4] == ref[4], mode


@pytest.mark.parametrize("waves,tile", [(1, 0), (4, 192)])
def test_step_path_equals_recomputed_path(waves, tile):
    """md_step_path keeps, from the state after step 0, bitwise the path that
    md_adjoint_recompute rebuilds from that state's checkpoint (positions in
    cell order with the user index, cell offsets), and ends on the state
    md_step reaches; md_adjoint_path over the kept path equals
    md_adjoint_segment from the checkpoint, bitwise, with one or four
    wavefronts per cell and the formula's or a 192-atom LDS tile."""
    torch = _torch()
    from paper_0709_3225_amd import _lib as L, LJSystem

    w = ljsynth.WORKLOADS["lj4k"]
    pos4, vel4, box = ljsynth.make_state(w, jitter_amp=0.05, shuffle=True)
    n, k = len(pos4), 7
    _say(f"step path vs recompute n={n} steps={k} waves={waves} tile={tile}")
    nc = LJSystem(n, box).cells_per_dim
    mk = lambda: (torch.empty((k, n, 4), dtype=torch.float32, device="cuda"),
                  torch.full((k, nc ** 3 + 1), -1, dtype=torch.int32, device="cuda"))
    a = LJSystem(n, box, dt=w.dt, waves_per_cell=waves, tile_cap=tile)
    a.load(_dev(pos4), _dev(vel4))
    cp, cv = a.state()
    cp, cv = cp.contiguous(), cv.contiguous()
    path_a, start_a = mk()
    L.md_step_path(a.params, a.ws, k, path_a, start_a)
    assert a.check() == 0
    b = LJSystem(n, box, dt=w.dt, waves_per_cell=waves, tile_cap=tile)
    path_b, start_b = mk()
    L.md_adjoint_recompute(b.params, b.ws, cp, cv, k, path_b, start_b)
    assert b.check() == 0
    assert torch.equal(start_a, start_b)
    assert torch.equal(path_a, path_b)
    # the workspace ends as after md_step
    c = LJSystem(n, box, dt=w.dt, waves_per_cell=waves, tile_cap=tile)
    c.load(_dev(pos4), _dev(vel4))
    c.step(k)
    pa, va = a.state()
    pc, vc = c.state()
    assert torch.equal(pa, pc) and torch.equal(va, vc)
    # the sweep over the kept path against the segment call
    rng = np.random.default_rng(12)
    lr0, lv0 = rng.standard_normal((n, 4)), rng.standard_normal((n, 4))
    out = []
    for kept in (True, False):
        lr, lv = _dev(lr0), _dev(lv0)
        th = torch.zeros(2, dtype=torch.float64, device="cuda")
        if kept:
            L.md_adjoint_path(a.params, a.ws, 2, k, path_a, start_a, lr, lv, th)
            assert a.check() == 0
        else:
            path, start = mk()
            L.md_adjoint_segment(b.params, b.ws, cp, cv, 2, k, path, start, lr, lv, th)
            assert b.check() == 0
        out.append((lr, lv, th))
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    assert torch.equal(out[0][2], out[1][2])
    # md_adjoint_path left the workspace's state in place
    pa2, va2 = a.state()
    assert torch.equal(pa, pa2) and torch.equal(va, va2)


@pytest.mark.parametrize("first_step", [0, 3])
def test_segment_equals_composed_calls(first_step):
    """md_adjoint_segment is the composition of the public calls it stands
    for, bitwise for the adjoint vectors: the states by md_build_cells +
    md_forces + md_step(1), and per step (last to first) md_adjoint_drift, then
    md_adjoint_kick on cells built from that state. The parameter gradient
    differs by FP64 summation order only. Afterwards the workspace holds no
    built state."""
    torch = _torch()
    from paper_0709_3225_amd import _lib as L, LJSystem, MDError

    w = ljsynth.WORKLOADS["lj4k"]
    pos4, vel4, box = ljsynth.make_state(w, jitter_amp=0.05)
    n, k = len(pos4), 6
    _say(f"segment vs composed calls n={n} steps={k} first_step={first_step}")
    s = LJSystem(n, box, dt=w.dt)
    h = 0.5 * w.dt
    rng = np.random.default_rng(7)
    lam_r0 = _dev(rng.standard_normal((n, 4)))
    lam_v0 = _dev(rng.standard_normal((n, 4)))
    cp, cv = _dev(pos4), _dev(vel4)
    # composed
    states = []
    L.md_build_cells(s.params, s.ws, cp, cv)
    L.md_forces(s.params, s.ws)
    for j in range(k):
        if j > 0:
            L.md_step(s.params, s.ws, 1)
        p_j = torch.empty((n, 4), dtype=torch.float32, device="cuda")
        L.md_get_state(s.params, s.ws, p_j, None)
        states.append(p_j)
    lr, lv = lam_r0.clone(), lam_v0.clone()
    th = torch.zeros(2, dtype=torch.float64, device="cuda")
    for j in range(k - 1, -1, -1):
        L.md_adjoint_drift(s.params, lr, lv)
        L.md_build_cells(s.params, s.ws, states[j], None)
        L.md_adjoint_kick(s.params, s.ws, lv, lr, th, 2 * h if first_step + j >= 1 else h)
    s.check()
    # one segment call
    nc, _ = L.md_cell_grid(s.params)
    path = torch.empty((k, n, 4), dtype=torch.float32, device="cuda")
    path_start = torch.empty((k, nc ** 3 + 1), dtype=torch.int32, device="cuda")
    sr, sv = lam_r0.clone(), lam_v0.clone()
    st = torch.zeros(2, dtype=torch.float64, device="cuda")
    L.md_adjoint_segment(s.params, s.ws, cp, cv, first_step, k, path, path_start, sr, sv, st)
    s.check()
    assert torch.equal(sr, lr) and torch.equal(sv, lv)
    # the segment sums the parameter terms per cell before the cells: FP64 order only
    assert torch.allclose(st, th, rtol=1e-12, atol=0.0)
    # the kept state j is the composed run's state j, cell-sorted
    for j in range(k):
        ids = path[j][:, 3].view(torch.int32).long()
        assert torch.equal(path[j][:, :3], states[j][ids, :3]), j
    L.md_forces(s.params, s.ws)
    with pytest.raises(MDError):
        s.check()
