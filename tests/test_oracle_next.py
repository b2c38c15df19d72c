"""Pins for the oracle on the widened workloads (CPU only): the WCA potential
(LJ truncated at its minimum 2^(1/6) sigma and shifted by eps, i.e. another
short-range pair potential as the paper's closing section allows) and LJ at
other densities (the density axis of the paper's cell-list measurements,
section 3.2).

The pins are closed forms and textbook lattice facts, not the oracle's own
formulas: the WCA energy at contact, lattices whose shells lie wholly inside
or outside the cutoff, and finite differences.
"""
import math

import numpy as np
import pytest

import ljsynth

RC_WCA = 2.0 ** (1.0 / 6.0)


def _wca(orc, box, eps=1.0, sig=1.0, mode=1):
    return orc.params(box, epsilon=eps, sigma=sig, rc=RC_WCA * sig, shift_mode=mode)


@pytest.mark.parametrize("eps,sig", [(1.0, 1.0), (0.6, 1.4)])
def test_wca_pair_closed_form(orc, eps, sig):
    """u_WCA(r) = 4 eps [(s/r)^12 - (s/r)^6] + eps below 2^(1/6) s, 0 beyond:
    u(s) = eps, u -> 0 and F -> 0 at the cutoff (the LJ minimum), F(s) =
    24 eps / s. The two shift modes agree, since f_LJ(r_c) = 0."""
    rc = RC_WCA * sig
    for mode in (0, 1):
        p = _wca(orc, 100.0, eps, sig, mode)
        phi_s, u_s = orc.pair(p, sig)
        assert u_s == pytest.approx(eps, rel=1e-12)
        assert phi_s == pytest.approx(24.0 * eps / sig, rel=1e-12)
        phi_in, u_in = orc.pair(p, rc * (1 - 1e-7))
        assert abs(phi_in) < 1e-5 * eps / sig and abs(u_in) < 1e-10 * eps
        assert orc.pair(p, rc * (1 + 1e-9)) == (0.0, 0.0)
        r = 0.93 * sig
        x = (sig / r) ** 6
        phi, u = orc.pair(p, r)
        assert u == pytest.approx(4 * eps * (x * x - x) + eps, rel=1e-12)
        assert phi == pytest.approx(24 * eps / r * (2 * x * x - x), rel=1e-12)


def test_wca_fcc_below_unit_density_is_free(orc):
    """FCC at rho <= 1 has nearest neighbours at (4/rho)^(1/3)/sqrt(2) >=
    2^(1/6): no pair interacts, so U = W = 0 and every force is zero."""
    w = ljsynth.WORKLOADS["lj4k"]  # rho = 0.8442
    L = ljsynth.box_length(w.n, w.density)
    pos = ljsynth.fcc_positions(w.n_fcc, L)
    assert L / w.n_fcc / math.sqrt(2.0) > RC_WCA
    f, U, W = orc.forces(_wca(orc, L), pos)
    assert U == 0.0 and W == 0.0 and np.abs(f).max() == 0.0


@pytest.mark.parametrize("mode", [0, 1])
def test_wca_fcc_first_shell(orc, mode):
    """FCC at rho = 1.2: the 12 nearest neighbours at a/sqrt(2) lie inside
    2^(1/6), the next shell (6 at a) outside, so U/N = 6 u(a/sqrt 2) and
    W/N = 6 (a/sqrt 2) phi(a/sqrt 2), with u and phi in closed form."""
    n_fcc, rho = 8, 1.2
    n = 4 * n_fcc ** 3
    L = ljsynth.box_length(n, rho)
    a = L / n_fcc
    r1 = a / math.sqrt(2.0)
    assert r1 < RC_WCA < a
    pos = ljsynth.fcc_positions(n_fcc, L)
    f, U, W = orc.forces(_wca(orc, L, mode=mode), pos)
    x = r1 ** -6
    u1 = 4 * (x * x - x) + 1.0
    phi1 = 24 / r1 * (2 * x * x - x)
    assert U / n == pytest.approx(6 * u1, rel=1e-10)
    assert W / n == pytest.approx(6 * r1 * phi1, rel=1e-9)
    assert np.abs(f).max() < 1e-9


def test_wca_force_is_minus_gradient(orc):
    n_fcc, rho = 5, 1.2
    n = 4 * n_fcc ** 3
    L = ljsynth.box_length(n, rho)
    pos = ljsynth.jitter(ljsynth.fcc_positions(n_fcc, L), 0.08, 11)
    p = _wca(orc, L)
    f, U, W = orc.forces(p, pos)
    assert np.abs(f).max() > 1.0  # the jitter makes pairs interact
    rng = np.random.default_rng(3)
    h = 1e-6
    for _ in range(10):
        i, c = int(rng.integers(n)), int(rng.integers(3))
        pp = pos.copy()
        pp[i, c] += h
        up = orc.forces(p, pp)[1]
        pp[i, c] -= 2 * h
        um = orc.forces(p, pp)[1]
        assert f[i, c] == pytest.approx(-(up - um) / (2 * h), rel=1e-5, abs=1e-6)


@pytest.mark.parametrize("rho,shells", [(0.2, [(1, 12)]), (0.5, [(1, 12), (2, 6), (3, 24)]),
                                        (1.0, [(1, 12), (2, 6), (3, 24), (4, 12)])])
def test_lj_fcc_shells_other_densities(orc, rho, shells):
    """LJ (r_c = 2.5) on FCC lattices at other densities: the shells
    a sqrt(k/2) inside r_c (multiplicities 12, 6, 24, 12 for k = 1..4)
    give U/N and W/N as half the shell sums; the net forces vanish."""
    n_fcc = 8
    n = 4 * n_fcc ** 3
    L = ljsynth.box_length(n, rho)
    a = L / n_fcc
    for k, _ in shells:
        assert a * math.sqrt(k / 2.0) < 2.5
    assert a * math.sqrt((len(shells) + 1) / 2.0) > 2.5  # the next shell is outside
    p = orc.params(L)
    pos = ljsynth.fcc_positions(n_fcc, L)
    f, U, W = orc.forces(p, pos)
    u_ref = w_ref = 0.0
    for k, z in shells:
        r = a * math.sqrt(k / 2.0)
        phi, u = orc.pair(p, r)
        u_ref += 0.5 * z * u
        w_ref += 0.5 * z * r * phi
    assert U / n == pytest.approx(u_ref, rel=1e-11)
    assert W / n == pytest.approx(w_ref, rel=1e-10)
    assert np.abs(f).max() < 1e-9
