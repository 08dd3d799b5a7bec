"""Pins of the oracle's self-consistent screening (range-separated SCS).

Each check ties the oracle to something other than itself:
- T_GG against a finite-difference Hessian of the Gaussian-cloud potential erf(r/sigma)/r;
- T_GG limits: the bare tensor far out, (4 / (3 sqrt(pi) sigma^3)) I at the centre;
- the frequency quadrature against the closed-form Casimir-Polder integral of one
  oscillator, C6 = (3/4) alpha^2 omega;
- an isolated atom is unscreened;
- a dimer against the closed form that symmetry gives: sum_j B_ij = (A^-1 + T)^-1;
- one atom per cubic cell: the image sum is isotropic, and equals a lattice sum written
  out independently;
- a supercell gives the same screened values per atom as its primitive cell.
"""
import itertools
import math

import numpy as np
import pytest
import torch

import synth
from oracle import scs as osc
from oracle import tensors as tz

A_B = synth.ANGSTROM_BOHR
BETA, DAMP = 0.83, 6.0


def _phi(x, sigma):
    r = math.sqrt(sum(c * c for c in x))
    return math.erf(r / sigma) / r


@pytest.mark.parametrize("rvec,sigma", [((1.3, -0.4, 2.2), 1.1), ((0.5, 0.6, -0.2), 1.7),
                                        ((3.0, 1.0, 0.5), 0.6)])
def test_gauss_tensor_is_minus_hessian_of_cloud_potential(rvec, sigma):
    h = 1e-3
    x0 = np.array(rvec)
    H = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            ea, eb = np.eye(3)[a] * h, np.eye(3)[b] * h
            H[a, b] = (_phi(x0 + ea + eb, sigma) - _phi(x0 + ea - eb, sigma)
                       - _phi(x0 - ea + eb, sigma) + _phi(x0 - ea - eb, sigma)) / (4 * h * h)
    r = torch.tensor(np.linalg.norm(x0), dtype=torch.float64)
    A, B = osc.radial_gauss(r, torch.tensor(sigma, dtype=torch.float64))
    T = float(A) * np.eye(3) - float(B) * np.outer(x0, x0)
    assert np.abs(T + H).max() < 1e-6 * np.abs(T).max()


def test_gauss_tensor_limits():
    sigma = torch.tensor(0.8, dtype=torch.float64)
    r = torch.tensor([12.0, 20.0], dtype=torch.float64)
    A, B = osc.radial_gauss(r, sigma)
    Ab, Bb = tz.radial_bare(r)
    assert torch.allclose(A, Ab, rtol=1e-14, atol=0) and torch.allclose(B, Bb, rtol=1e-14, atol=0)
    # inside the cloud the field of a Gaussian dipole is uniform: 4 / (3 sqrt(pi) sigma^3)
    r0 = 1e-3 * sigma
    A0, B0 = osc.radial_gauss(r0, sigma)
    assert float(A0) == pytest.approx(4.0 / (3.0 * math.sqrt(math.pi) * float(sigma) ** 3),
                                      rel=1e-5)
    assert abs(float(B0 * r0 * r0)) < 1e-5 * float(A0)


@pytest.mark.parametrize("n,tol", [(15, 3e-8), (20, 5e-11)])
def test_freq_grid_gives_one_oscillator_c6(n, tol):
    u, w = osc.freq_grid(n)
    assert float((w / (1.0 + u * u)).sum()) == pytest.approx(math.pi / 2, rel=1e-6)
    for alpha, omega in [(10.0, 0.2), (5.0, 0.5), (12.0, 1.5)]:
        au = osc.alpha_dynamic(alpha, omega, u)
        c6 = 3.0 / math.pi * float((w * au * au).sum())
        assert c6 == pytest.approx(0.75 * alpha * alpha * omega, rel=tol)


def test_isolated_atom_is_unscreened():
    s = synth.one_atom(alpha=9.0, omega=0.45, rvdw=3.4, L_ang=40.0)
    a0, om, rv, u, au = osc.scs(s, BETA, DAMP, rcut=12.0 * A_B)
    assert float(a0[0]) == pytest.approx(9.0, rel=1e-14)
    assert torch.allclose(au[:, 0], torch.as_tensor(osc.alpha_dynamic(9.0, 0.45, u)),
                          rtol=1e-14, atol=0)
    assert float(om[0]) == pytest.approx(0.45, rel=1e-8)
    assert float(rv[0]) == pytest.approx(3.4, rel=1e-14)


@pytest.mark.parametrize("r_ang,u", [(2.5, 0.0), (3.2, 0.0), (3.2, 0.7)])
def test_dimer_matches_symmetry_closed_form(r_ang, u):
    s = synth.dimer(r_ang, L_ang=60.0, alpha=9.0, omega=0.5, rvdw=3.3)
    got = osc.screened_alpha(s, u, BETA, DAMP, rcut=15.0 * A_B)
    a = osc.alpha_dynamic(9.0, 0.5, u)
    r = torch.tensor(r_ang * A_B, dtype=torch.float64)
    Ag, Bg = osc.radial_gauss(r, math.sqrt(2.0) * osc.gaussian_sigma(a))
    g = float(tz.one_minus_fermi(r, BETA * 6.6, DAMP))
    t_perp, t_par = g * float(Ag), g * float(Ag - Bg * r * r)
    want = (2.0 * a / (1.0 + a * t_perp) + a / (1.0 + a * t_par)) / 3.0
    assert torch.allclose(got, torch.tensor([want, want], dtype=torch.float64), rtol=1e-13, atol=0)
    assert t_par < 0.0 < t_perp  # head-to-tail enhances, side-by-side depolarizes


def test_one_atom_per_cubic_cell_lattice_sum():
    a_ang = 3.0
    s = synth.simple_cubic(1, a_ang, alpha=7.0, omega=0.5, rvdw=3.0)
    rc = 14.0 * A_B
    M = osc.screening_matrix(s, 0.0, BETA, DAMP, rc)
    assert float((M - torch.diag(torch.diagonal(M))).abs().max()) < 1e-14 * float(M.abs().max())
    assert float(M[0, 0]) == pytest.approx(float(M[1, 1]), rel=1e-13)
    # the same lattice sum written out: (1/3) tr T_SR(n) = (1 - f)(3A - B r^2)/3
    L = a_ang * A_B
    sig = math.sqrt(2.0) * osc.gaussian_sigma(7.0)
    t = 0.0
    nmax = int(rc / L) + 1
    for n in itertools.product(range(-nmax, nmax + 1), repeat=3):
        r = L * math.sqrt(n[0] ** 2 + n[1] ** 2 + n[2] ** 2)
        if r == 0.0 or r >= rc:
            continue
        z = r / sig
        c = 2.0 / math.sqrt(math.pi) * z * math.exp(-z * z)
        Ag = (math.erf(z) - c) / r ** 3
        Bg = (3.0 * math.erf(z) - c * (3.0 + 2.0 * z * z)) / r ** 5
        g = 1.0 / (1.0 + math.exp(DAMP * (r / (BETA * 6.0) - 1.0)))
        t += g * (3.0 * Ag - Bg * r * r) / 3.0
    assert float(M[0, 0]) - 1.0 / 7.0 == pytest.approx(t, rel=1e-12)
    a0 = osc.screened_alpha(s, 0.0, BETA, DAMP, rc)
    assert float(a0[0]) == pytest.approx(7.0 / (1.0 + 7.0 * t), rel=1e-12)


def test_supercell_gives_the_same_screening():
    s = synth.tiny_random(seed=3, n=20, L_ang=7.0, dmin_ang=2.2)
    two = synth.System("x2", np.concatenate([s.pos, s.pos + s.cell[0]]),
                       s.cell * np.array([[2.0], [1.0], [1.0]]),
                       np.tile(s.alpha, 2), np.tile(s.omega, 2), np.tile(s.rvdw, 2))
    rc = 9.0 * A_B
    a1, o1, r1, _, _ = osc.scs(s, BETA, DAMP, rc, n_freq=6)
    a2, o2, r2, _, _ = osc.scs(two, BETA, DAMP, rc, n_freq=6)
    for x, y in [(a1, a2), (o1, o2), (r1, r2)]:
        assert torch.allclose(torch.cat([x, x]), y, rtol=1e-11, atol=0)


def test_screening_is_translation_and_permutation_invariant():
    s = synth.tiny_random(seed=5, n=24, L_ang=7.5, dmin_ang=2.2)
    rc = 9.0 * A_B
    base = osc.screened_alpha(s, 0.3, BETA, DAMP, rc)
    perm = np.random.default_rng(1).permutation(s.n)
    moved = synth.System("t", s.pos[perm] + np.array([3.1, -7.7, 40.2]), s.cell, s.alpha[perm],
                         s.omega[perm], s.rvdw[perm])
    got = osc.screened_alpha(moved, 0.3, BETA, DAMP, rc)
    assert torch.allclose(got, base[perm], rtol=1e-11, atol=0)
