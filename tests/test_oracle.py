"""Pins for the FP64 reference oracle (CPU only).

Each test fixes part of the oracle against something other than the oracle's
own formulas: textbook LJ facts, the paper's statements (section 2: force
shifted to zero at the cutoff, sign of the force sum), exact scaling laws,
finite differences, lattice sums over textbook FCC shells, invariances,
brute force on tiny inputs, and properties of velocity Verlet.
"""
import json
import math
import os

import numpy as np
import pytest

import ljsynth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _p(orc, box, **kw):
    return orc.params(box, **kw)


# ---------------------------------------------------------------- pair terms

@pytest.mark.parametrize("eps,sig", [(1.0, 1.0), (0.7, 1.3), (2.0, 0.8)])
def test_pair_textbook_points(orc, eps, sig):
    """LJ facts: F(sigma) = 24 eps / sigma, F = 0 at the minimum 2^(1/6) sigma,
    well depth u(r_min) - u(sigma) = -eps (shift cancels in differences).
    Energy-shift mode leaves the force unshifted."""
    p = _p(orc, 100.0, epsilon=eps, sigma=sig, shift_mode=1)
    rmin = 2.0 ** (1.0 / 6.0) * sig
    phi_min, u_min = orc.pair(p, rmin)
    phi_s, u_s = orc.pair(p, sig)
    assert abs(phi_min) < 1e-12 * eps / sig
    assert phi_s == pytest.approx(24.0 * eps / sig, rel=1e-13)
    assert u_min - u_s == pytest.approx(-eps, rel=1e-13)


@pytest.mark.parametrize("mode", [0, 1])
def test_pair_zero_at_cutoff(orc, mode):
    """Section 2: the force is shifted to vanish at r_c = 2.5 sigma; it is zero
    beyond. The matching energy is continuous there (zero at r_c)."""
    p = _p(orc, 100.0, epsilon=1.3, sigma=0.9, shift_mode=mode)
    rc = 2.5 * 0.9
    phi_in, u_in = orc.pair(p, rc * (1 - 1e-9))
    phi_out, u_out = orc.pair(p, rc * (1 + 1e-9))
    assert phi_out == 0.0 and u_out == 0.0
    assert abs(u_in) < 1e-9
    if mode == 0:
        assert abs(phi_in) < 1e-8
    phi_at, u_at = orc.pair(p, rc)  # strict cutoff: r = r_c does not interact
    assert phi_at == 0.0 and u_at == 0.0


def test_force_shift_is_constant_offset(orc):
    """f(r) = f_LJ(r) - f_LJ(r_c): the two modes differ by one constant."""
    p0 = _p(orc, 100.0, epsilon=1.1, sigma=1.2, shift_mode=0)
    p1 = _p(orc, 100.0, epsilon=1.1, sigma=1.2, shift_mode=1)
    rs = np.linspace(0.9, 2.99, 37)
    diffs = [orc.pair(p0, r)[0] - orc.pair(p1, r)[0] for r in rs]
    assert np.ptp(diffs) < 1e-12
    # the constant is -f_LJ(r_c), and f_LJ(r_c) < 0 (attractive at 2.5 sigma)
    assert diffs[0] > 0


@pytest.mark.parametrize("mode", [0, 1])
def test_pair_force_is_minus_energy_derivative(orc, mode):
    p = _p(orc, 100.0, epsilon=0.8, sigma=1.1, shift_mode=mode)
    for r in [0.95, 1.05, 1.2347, 1.6, 2.0, 2.6]:
        h = 1e-6
        du = (orc.pair(p, r + h)[1] - orc.pair(p, r - h)[1]) / (2 * h)
        assert orc.pair(p, r)[0] == pytest.approx(-du, rel=1e-7, abs=1e-9)


def test_pair_scaling_law(orc):
    """u(r; eps, sigma) = eps u(r/sigma; 1, 1) and, through F = -du/dr,
    F(r; eps, sigma) = (eps/sigma) F(r/sigma; 1, 1). This fixes the 1/sigma
    factor the paper's printed f_LJ omits."""
    p1 = _p(orc, 100.0)
    eps, sig = 1.7, 1.35
    ps = _p(orc, 100.0, epsilon=eps, sigma=sig)
    for x in [0.93, 1.1, 1.5, 2.2, 2.49]:
        phi1, u1 = orc.pair(p1, x)
        phis, us = orc.pair(ps, x * sig)
        assert us == pytest.approx(eps * u1, rel=1e-12, abs=1e-15)
        assert phis == pytest.approx(eps / sig * phi1, rel=1e-12, abs=1e-15)


# ------------------------------------------------------------- small systems

def test_two_atoms_sign_and_images(orc):
    """Section 2 force sum: positive f pushes the pair apart. Checked directly
    and across the periodic boundary (minimum image)."""
    L = 10.0
    p = _p(orc, L)
    pos = np.array([[1.0, 5.0, 5.0], [2.0, 5.0, 5.0]])
    f, U, W = orc.forces(p, pos)
    phi, u = orc.pair(p, 1.0)
    assert phi > 0
    np.testing.assert_allclose(f, [[-phi, 0, 0], [phi, 0, 0]], rtol=1e-14, atol=1e-14)
    assert U == pytest.approx(u, rel=1e-14)
    assert W == pytest.approx(1.0 * phi, rel=1e-14)
    # across the boundary: 0.2 and 9.3 are 0.9 apart through x = 0
    pos = np.array([[0.2, 5.0, 5.0], [9.3, 5.0, 5.0]])
    f, U, W = orc.forces(p, pos)
    phi, u = orc.pair(p, 0.9)
    np.testing.assert_allclose(f, [[phi, 0, 0], [-phi, 0, 0]], rtol=1e-12, atol=1e-12)
    # beyond the cutoff nothing acts
    pos = np.array([[1.0, 1.0, 1.0], [1.0, 1.0, 3.6]])
    f, U, W = orc.forces(p, pos)
    assert np.all(f == 0) and U == 0 and W == 0


def test_three_collinear_atoms(orc):
    L = 20.0
    p = _p(orc, L)
    pos = np.array([[3.0, 4.0, 4.0], [4.0, 4.0, 4.0], [5.2, 4.0, 4.0]])
    f, U, W = orc.forces(p, pos)
    a, ua = orc.pair(p, 1.0)
    b, ub = orc.pair(p, 2.2)
    c, uc = orc.pair(p, 1.2)
    np.testing.assert_allclose(f[:, 0], [-(a + b), a - c, b + c], rtol=1e-12)
    np.testing.assert_allclose(f[:, 1:], 0, atol=1e-15)
    assert U == pytest.approx(ua + ub + uc, rel=1e-13)
    assert W == pytest.approx(1.0 * a + 2.2 * b + 1.2 * c, rel=1e-13)


def test_single_atom_has_no_force(orc):
    f, U, W = orc.forces(_p(orc, 6.0), np.array([[1.0, 2.0, 3.0]]))
    assert np.all(f == 0) and U == 0 and W == 0


def test_box_too_small_rejected(orc):
    with pytest.raises(ValueError):
        orc.forces(_p(orc, 4.9), np.zeros((2, 3)))


# -------------------------------------------------------------- lattice sums

@pytest.mark.parametrize("mode", [0, 1])
def test_fcc_lattice_sum(orc, mode):
    """Perfect FCC at rho = 0.8442: every atom sees textbook shells
    a sqrt(k/2) with multiplicities 12, 6, 24, 12 inside r_c = 2.5, so
    U/N = 1/2 sum z_k u(r_k) and W/N = 1/2 sum z_k r_k phi(r_k), and the net
    force on every atom vanishes by symmetry."""
    shells = json.load(open(os.path.join(GOLDEN, "fcc_shells.json")))["shells"]
    w = ljsynth.WORKLOADS["lj4k"]
    L = ljsynth.box_length(w.n, w.density)
    a = L / w.n_fcc
    p = _p(orc, L, shift_mode=mode)
    pos = ljsynth.fcc_positions(w.n_fcc, L)  # FP64 lattice (no FP32 rounding)
    f, U, W = orc.forces(p, pos)
    u_ref = w_ref = 0.0
    inside = 0
    for k, z in shells:
        r = a * math.sqrt(k / 2.0)
        if r < 2.5:
            phi, u = orc.pair(p, r)
            u_ref += 0.5 * z * u
            w_ref += 0.5 * z * r * phi
            inside += z
    assert inside == 54
    assert U / w.n == pytest.approx(u_ref, rel=1e-12)
    assert W / w.n == pytest.approx(w_ref, rel=1e-12)
    assert np.abs(f).max() < 1e-10
    if mode == 0:
        # value recomputed in FP64 from the same shells (force-shift energy)
        assert U / w.n == pytest.approx(-5.693278, abs=2e-6)
        assert W / w.n == pytest.approx(-20.16527, abs=2e-5)


# --------------------------------------------------- gradients and identities

def _jittered(w, amp=0.05):
    pos4, vel4, L = ljsynth.make_state(w, jitter_amp=amp)
    return pos4[:, :3].astype(np.float64), vel4[:, :3].astype(np.float64), L


def test_newton_third_law(orc):
    pos, _, L = _jittered(ljsynth.WORKLOADS["lj4k"])
    f, U, W = orc.forces(_p(orc, L), pos)
    assert np.abs(f.sum(axis=0)).max() < 1e-11 * np.abs(f).max() * len(f) ** 0.5


@pytest.mark.parametrize("mode", [0, 1])
def test_force_is_minus_gradient(orc, mode):
    pos, _, L = _jittered(ljsynth.WORKLOADS["lj256_check"], amp=0.1)
    p = _p(orc, L, shift_mode=mode)
    f, U, W = orc.forces(p, pos)
    rng = np.random.default_rng(7)
    h = 1e-5
    for _ in range(12):
        i = int(rng.integers(len(pos)))
        c = int(rng.integers(3))
        pp = pos.copy()
        pp[i, c] += h
        up = orc.forces(p, pp)[1]
        pp[i, c] -= 2 * h
        um = orc.forces(p, pp)[1]
        fd = -(up - um) / (2 * h)
        assert f[i, c] == pytest.approx(fd, rel=1e-6, abs=1e-7)


def test_virial_is_volume_derivative(orc):
    """Uniform dilation r -> lam r, L -> lam L: dU/dlam at lam = 1 is -W."""
    pos, _, L = _jittered(ljsynth.WORKLOADS["lj256_check"], amp=0.1)
    h = 1e-6
    _, U, W = orc.forces(_p(orc, L), pos)
    up = orc.forces(_p(orc, L * (1 + h)), pos * (1 + h))[1]
    um = orc.forces(_p(orc, L * (1 - h)), pos * (1 - h))[1]
    assert -(up - um) / (2 * h) == pytest.approx(W, rel=1e-7)


@pytest.mark.parametrize("mode", [0, 1])
def test_euler_identities(orc, mode):
    """U = eps Phi(r/sigma) with r_c = 2.5 sigma gives eps dU/deps = U and
    sigma dU/dsigma = W (no boundary term: u(r_c) = 0)."""
    pos, _, L = _jittered(ljsynth.WORKLOADS["lj256_check"], amp=0.1)
    eps, sig, h = 1.0, 1.0, 1e-6
    _, U, W = orc.forces(_p(orc, L, shift_mode=mode), pos)
    ue = [orc.forces(_p(orc, L, epsilon=eps * (1 + s * h), shift_mode=mode), pos)[1] for s in (1, -1)]
    us = [orc.forces(_p(orc, L, sigma=sig * (1 + s * h), shift_mode=mode), pos)[1] for s in (1, -1)]
    assert (ue[0] - ue[1]) / (2 * h) == pytest.approx(U, rel=1e-7)
    assert (us[0] - us[1]) / (2 * h) == pytest.approx(W, rel=1e-6)


def test_translation_and_permutation(orc):
    pos, _, L = _jittered(ljsynth.WORKLOADS["lj256_check"], amp=0.1)
    p = _p(orc, L)
    f, U, W = orc.forces(p, pos)
    shifted = np.mod(pos + np.array([0.37, -1.2, 2.9]), L)
    f2, U2, W2 = orc.forces(p, shifted)
    np.testing.assert_allclose(f2, f, rtol=1e-9, atol=1e-9)
    assert U2 == pytest.approx(U, rel=1e-11)
    perm = np.random.default_rng(3).permutation(len(pos))
    f3, U3, W3 = orc.forces(p, pos[perm])
    np.testing.assert_allclose(f3, f[perm], rtol=1e-11, atol=1e-11)
    assert W3 == pytest.approx(W, rel=1e-12)


def test_rows_match_full(orc):
    pos, _, L = _jittered(ljsynth.WORKLOADS["lj256_check"], amp=0.1)
    p = _p(orc, L)
    f, U, W = orc.forces(p, pos)
    rows = np.array([5, 0, 255, 17])
    fr, ur, wr = orc.forces_rows(p, pos, rows)
    np.testing.assert_array_equal(fr, f[rows])
    fa, ua, wa = orc.forces_rows(p, pos, np.arange(len(pos)))
    assert ua.sum() == pytest.approx(U, rel=1e-13)
    assert wa.sum() == pytest.approx(W, rel=1e-13)


def test_kinetic(orc):
    v = np.array([[1.0, 2.0, 2.0], [0.0, 0.0, -1.0]])
    assert orc.kinetic(_p(orc, 10.0, mass=2.0), v) == pytest.approx(0.5 * 2.0 * (9 + 1))


# ------------------------------------------------------------------ neighbours

def test_neighbors_brute_force(orc):
    rng = np.random.default_rng(11)
    L = 6.0
    pos = rng.uniform(0, L, size=(40, 3))
    p = _p(orc, L)
    counts, idx, guard = orc.neighbors(p, pos)
    off = np.concatenate([[0], np.cumsum(counts)])
    for i in range(len(pos)):
        expect = []
        for j in range(len(pos)):
            if i == j:
                continue
            d = pos[i] - pos[j]
            d = d - L * np.round(d / L)
            if (d * d).sum() < 6.25:
                expect.append(j)
        assert list(idx[off[i]:off[i + 1]]) == expect


def _lattice_neighbor_sets(pos, box, n_fcc, d2_max):
    """Neighbour sets of a perfect FCC lattice by integer arithmetic: site
    coordinates in units of half the lattice constant are integers (the
    common a/4 offset drops out of every difference), the minimum image is
    taken modulo 2 n_fcc, and shell k of the lattice lies at squared integer
    distance 2 k."""
    a = box / n_fcc
    g = np.rint((np.asarray(pos, np.float64)[:, :3] / a - 0.25) * 2.0).astype(np.int64) % (2 * n_fcc)
    d = g[:, None, :] - g[None, :, :]
    d = (d + n_fcc) % (2 * n_fcc) - n_fcc
    d2 = (d * d).sum(-1)
    np.fill_diagonal(d2, 1 << 30)
    return [np.flatnonzero(row <= d2_max) for row in d2]


@pytest.mark.parametrize("density,n_fcc,shells", [(0.8442, 10, 4), (0.5, 6, 3)])
def test_neighbors_of_perfect_fcc(orc, density, n_fcc, shells):
    """On a perfect FCC lattice every atom has the same neighbours: the sites
    of the textbook shells inside r_c = 2.5 (at rho = 0.8442, a = 1.6796: the
    first four shells, 12 + 6 + 24 + 12 = 54 sites, the fifth at 2.656 is
    outside; at rho = 0.5, a = 2: three shells, 42 sites). The oracle's
    brute-force sets must equal the sets found by integer lattice arithmetic,
    site for site."""
    g = json.load(open(os.path.join(GOLDEN, "fcc_shells.json")))
    expect = sum(m for k, m in g["shells"][:shells])
    w = ljsynth.Workload("fcc", n_fcc, density, 1.0, 1, 1)
    pos, _, L = ljsynth.make_state(w)
    a = L / n_fcc
    assert a * math.sqrt(shells / 2.0) < 2.5 < a * math.sqrt((shells + 1) / 2.0)
    counts, idx, guard = orc.neighbors(_p(orc, L), pos)
    assert guard == 0
    assert np.all(counts == expect)
    lattice = _lattice_neighbor_sets(pos, L, n_fcc, 2 * shells)
    off = np.concatenate([[0], np.cumsum(counts)])
    for i in range(len(pos)):
        assert np.array_equal(idx[off[i]:off[i + 1]], lattice[i]), i


def test_guard_band_empty_for_parity_state(orc):
    pos, _, L = _jittered(ljsynth.WORKLOADS["lj4k"])
    counts, idx, guard = orc.neighbors(_p(orc, L), pos)
    assert guard == 0
    assert 50 < counts.mean() < 60  # about 4/3 pi rho r_c^3 = 55.25


# ------------------------------------------------------------------ integrator

def test_verlet_time_reversible(orc):
    """Velocity Verlet is time reversible: run forward, flip velocities, run
    the same number of steps, and the start state returns (up to rounding)."""
    pos, vel, L = _jittered(ljsynth.WORKLOADS["lj256_check"], amp=0.02)
    p = _p(orc, L)
    x1, v1, _ = orc.run(p, pos, vel, 20)
    x2, v2, _ = orc.run(p, x1, -v1, 20)
    d = x2 - pos
    d -= L * np.round(d / L)
    assert np.abs(d).max() < 1e-9
    np.testing.assert_allclose(-v2, vel, atol=1e-9)


def test_verlet_momentum_and_energy(orc):
    """The N = 4000 parity workload, 100 NVE steps at dt = 0.005 from the
    lattice: total energy stays within 5e-4 relative of its start (the
    velocity-Verlet excursion, about 1.8e-4 here, scales as dt^2, which
    test_verlet_second_order pins) and momentum is conserved."""
    w = ljsynth.WORKLOADS["lj4k"]
    pos, vel, L = _jittered(w, amp=0.0)
    p = _p(orc, L)
    x, v, th = orc.run(p, pos, vel, 100)
    e = th[:, 0] + th[:, 1]
    assert np.abs(e - e[0]).max() / abs(e[0]) < 5e-4
    np.testing.assert_allclose(v.sum(axis=0), vel.sum(axis=0), atol=1e-10)


def test_verlet_second_order(orc):
    """Energy error of velocity Verlet scales as dt^2: halving dt over the
    same simulated time cuts the largest energy excursion about fourfold."""
    pos, vel, L = _jittered(ljsynth.WORKLOADS["lj256_check"], amp=0.02)
    errs = []
    for dt, n in [(0.004, 25), (0.002, 50)]:
        _, _, th = orc.run(_p(orc, L, dt=dt), pos, vel, n)
        e = th[:, 0] + th[:, 1]
        errs.append(np.abs(e - e[0]).max())
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_paper_worked_example_golden_is_consistent():
    """The section 3.2 example: int(11/2.5) = 4 cells of side 2.75; the cell
    volume ratio 1.1^3 and its square match the quoted 33% and 77%."""
    g = json.load(open(os.path.join(GOLDEN, "paper_cell_example.json")))
    assert int(g["box"] / g["rc"]) == g["cells_per_dim"]
    assert g["box"] / g["cells_per_dim"] == g["cell_side"]
    ratio = (g["cell_side"] / g["rc"]) ** 3
    assert round(100 * (ratio - 1)) == g["particles_per_cell_increase_pct"]
    assert round(100 * (ratio ** 2 - 1)) == g["interactions_increase_pct"]


def test_full_size_energy_golden_is_consistent(orc):
    """The stored full O(N^2) oracle sums of the jittered N = 256,000 state
    (tests/golden/make_full_energy.py) against an independent estimate: the
    mean of 4,096 uniformly sampled rows, each a full sum over all N atoms,
    times N (a statistical check, 1e-3), and the recorded box and recipe."""
    g = json.load(open(os.path.join(GOLDEN, "lj256k_jitter_energy.json")))
    w = ljsynth.WORKLOADS["lj256k"]
    pos, _, L = ljsynth.make_state(w, jitter_amp=g["jitter"])
    assert g["n"] == w.n and g["seed"] == w.seed and g["box"] == L
    rows = np.random.default_rng(3).choice(w.n, size=4096, replace=False)
    _, ur, wr = orc.forces_rows(_p(orc, L), pos, rows)
    assert ur.mean() * w.n == pytest.approx(g["U"], rel=1e-3)
    assert wr.mean() * w.n == pytest.approx(g["W"], rel=1e-3)
