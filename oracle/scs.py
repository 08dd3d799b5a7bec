"""Self-consistent screening of the polarizabilities (oracle), range-separated form.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The Review section describes the MBD@rsSCS pipeline: the atom-in-molecule
polarizabilities are made frequency dependent, a Dyson-like screening equation
is solved at a set of imaginary frequencies, and the screened quantities enter
the MBD matrix. The paper does not write the screening equation out; the
readings taken here are those of the range-separated SCS of MBD@rsSCS:

- dynamic polarizability of one oscillator: alpha_i(iu) = alpha_i / (1 + (u / omega_i)^2);
- Gaussian width of the dipole's charge cloud: sigma_i(u) = (sqrt(2/pi) alpha_i(iu) / 3)^(1/3),
  and sigma_ij = sqrt(sigma_i^2 + sigma_j^2) for a pair;
- screening tensor T_SR = (1 - f) T_GG, with T_GG = -grad grad (erf(r / sigma_ij) / r) the
  dipole tensor between Gaussian charge clouds and f the Fermi damping of the MBD step
  (same beta, d and unscreened R_vdW). 1 - f makes it short-ranged: in a periodic cell it is
  summed over every image within the pair cutoff, with no Ewald split;
- screened polarizability: alpha^SCS_i(iu) = (1/3) tr sum_j [(A(iu)^-1 + T_SR(iu))^-1]_ij
  with A(iu) = diag(alpha_i(iu)) (x) I_3 (energy convention for T, as in the MBD matrix);
- C6^SCS_i = (3/pi) int_0^inf alpha^SCS_i(iu)^2 du (Casimir-Polder), by Gauss-Legendre
  quadrature mapped to [0, inf) with u = L (1 + x) / (1 - x);
- omega^SCS_i = 4 C6^SCS_i / (3 alpha^SCS_i(0)^2) (the one-oscillator relation
  C6 = (3/4) alpha^2 omega solved for omega), R^SCS_i = R_i (alpha^SCS_i(0) / alpha_i)^(1/3).

Everything is dense float64 linear algebra on the definition: for small systems only.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import tensors as tz

SQRTPI = math.sqrt(math.pi)


def alpha_dynamic(alpha, omega, u):
    """alpha(iu) of one harmonic oscillator with static alpha and frequency omega."""
    return alpha / (1.0 + (u / omega) ** 2)


def gaussian_sigma(alpha_u):
    """Width of the Gaussian charge cloud of a dipole with polarizability alpha_u."""
    return (math.sqrt(2.0 / math.pi) * alpha_u / 3.0) ** (1.0 / 3.0)


def radial_gauss(r, sigma):
    """T_GG = -grad grad (erf(r / sigma) / r) as (A, B), T = A I - B r r^T.

    With z = r / sigma and c = (2 / sqrt(pi)) z exp(-z^2):
    A = (erf(z) - c) / r^3,  B = (3 erf(z) - c (3 + 2 z^2)) / r^5."""
    z = r / sigma
    c = 2.0 / SQRTPI * z * torch.exp(-z * z)
    er = torch.special.erf(z)
    r2 = r * r
    r3 = r2 * r
    return (er - c) / r3, (3.0 * er - c * (3.0 + 2.0 * z * z)) / (r3 * r2)


def freq_grid(n: int, L: float = 0.6):
    """Nodes u_q and weights w_q with sum_q w_q g(u_q) ~ int_0^inf g(u) du: n-point
    Gauss-Legendre on x in (-1, 1) mapped by u = L (1 + x) / (1 - x)."""
    x, w = np.polynomial.legendre.leggauss(n)
    u = L * (1.0 + x) / (1.0 - x)
    return u, w * 2.0 * L / (1.0 - x) ** 2


def screening_matrix(sys, u: float, beta: float, d: float, rcut: float):
    """Dense M(iu) = A(iu)^-1 + T_SR(iu), 3N x 3N, pairs (i, j, n) within rcut."""
    pos = torch.as_tensor(sys.pos, dtype=torch.float64)
    N = pos.shape[0]
    al = torch.as_tensor(sys.alpha, dtype=torch.float64)
    om = torch.as_tensor(sys.omega, dtype=torch.float64)
    rv = torch.as_tensor(sys.rvdw, dtype=torch.float64)
    au = alpha_dynamic(al, om, u)
    sig = gaussian_sigma(au)
    i, j, r = tz.pair_list_bruteforce(pos, sys.cell, rcut)
    rn = torch.sqrt((r * r).sum(-1))
    A, B = radial_gauss(rn, torch.sqrt(sig[i] ** 2 + sig[j] ** 2))
    g = tz.one_minus_fermi(rn, beta * (rv[i] + rv[j]), d)
    blocks = (g * A)[:, None, None] * torch.eye(3, dtype=torch.float64) \
        - (g * B)[:, None, None] * r[:, :, None] * r[:, None, :]
    T = torch.zeros(N * N, 3, 3, dtype=torch.float64).index_add_(0, i * N + j, blocks)
    M = T.reshape(N, N, 3, 3).permute(0, 2, 1, 3).reshape(3 * N, 3 * N)
    return M + torch.diag((1.0 / au).repeat_interleave(3))


def screened_alpha(sys, u: float, beta: float, d: float, rcut: float):
    """alpha^SCS_i(iu) = (1/3) tr sum_j B_ij with B = M(iu)^-1."""
    N = len(sys.alpha)
    Binv = torch.linalg.inv(screening_matrix(sys, u, beta, d, rcut))
    blk = Binv.reshape(N, 3, N, 3).sum(2)
    return torch.diagonal(blk, dim1=1, dim2=2).sum(-1) / 3.0


def scs(sys, beta: float, d: float, rcut: float, n_freq: int = 15, L: float = 0.6):
    """Screened (alpha(0), omega, R_vdW) per atom, and alpha^SCS at every node.

    Returns alpha0 [N], omega [N], rvdw [N], nodes u [n_freq], alpha_u [n_freq][N]."""
    u, w = freq_grid(n_freq, L)
    a0 = screened_alpha(sys, 0.0, beta, d, rcut)
    au = torch.stack([screened_alpha(sys, float(x), beta, d, rcut) for x in u])
    c6 = 3.0 / math.pi * (torch.as_tensor(w)[:, None] * au * au).sum(0)
    om = 4.0 * c6 / (3.0 * a0 * a0)
    rv = torch.as_tensor(sys.rvdw, dtype=torch.float64) * \
        (a0 / torch.as_tensor(sys.alpha, dtype=torch.float64)) ** (1.0 / 3.0)
    return a0, om, rv, u, au
