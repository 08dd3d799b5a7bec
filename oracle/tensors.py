"""Dipole interaction tensors and real-space pair sums (oracle).

Every isotropic dipole tensor used here has the form T(r) = A(r) I - B(r) r r^T:

- bare dipole tensor  T = -grad grad (1/r):       A = 1/r^3, B = 3/r^5
- erfc-screened part  T_erfc = -grad grad (erfc(tau r)/r), the direct-space
  Ewald kernel (eq. fld_ewald):
      A = [erfc(x) + (2x/sqrt(pi)) e^{-x^2}] / r^3
      B = [3 erfc(x) + (2x/sqrt(pi)) (3 + 2x^2) e^{-x^2}] / r^5,   x = tau r
- damped tensor T' = f T (Review section: T' = s(R; beta) T) with the
  Fermi damping f(r) = 1 / (1 + exp(-d (r / S - 1))), S = beta (R_i + R_j).
  The paper defers the explicit damping to its stochastic-MBD reference; the
  Fermi form with the rsSCS range parameter beta and steepness d is the
  reading taken here.

Direct-space Ewald kernel with damping (eq. fld_ewald, read as a sum over all
images of the erfc part plus the damping correction): T_dir = T_erfc - (1-f) T.
1 - f is evaluated directly as 1 / (1 + exp(d (r/S - 1))).
"""
from __future__ import annotations

import math

import numpy as np
import torch

SQRTPI = math.sqrt(math.pi)


def radial_bare(r):
    r2 = r * r
    r3 = r2 * r
    return 1.0 / r3, 3.0 / (r3 * r2)


def radial_erfc(r, tau):
    x = tau * r
    ex = torch.exp(-x * x)
    c = 2.0 * x / SQRTPI * ex
    ec = torch.special.erfc(x)
    r2 = r * r
    r3 = r2 * r
    A = (ec + c) / r3
    B = (3.0 * ec + c * (3.0 + 2.0 * x * x)) / (r3 * r2)
    return A, B


def one_minus_fermi(r, S, d):
    return 1.0 / (1.0 + torch.exp(d * (r / S - 1.0)))


def fermi(r, S, d):
    return 1.0 / (1.0 + torch.exp(-d * (r / S - 1.0)))


def radial_direct(r, tau, S, d):
    """T_erfc - (1 - f) T_bare as (A, B)."""
    Ae, Be = radial_erfc(r, tau)
    Ab, Bb = radial_bare(r)
    g = one_minus_fermi(r, S, d)
    return Ae - g * Ab, Be - g * Bb


def radial_damped(r, S, d):
    """Free-space damped tensor f T as (A, B)."""
    Ab, Bb = radial_bare(r)
    f = fermi(r, S, d)
    return f * Ab, f * Bb


def apply_pairs(A, B, rvec, dsrc):
    """Field contributions T(r) d for a list of pairs: A d - B r (r . d).

    rvec: (P, 3); dsrc: (P, 3, nrhs). Returns (P, 3, nrhs).
    """
    rd = torch.einsum("pc,pcb->pb", rvec, dsrc)
    return A[:, None, None] * dsrc - B[:, None, None] * rvec[:, :, None] * rd[:, None, :]


def image_range(cell: np.ndarray, rc: float) -> np.ndarray:
    """Integer range n_max per axis so that every image within rc of any
    in-cell displacement is enumerated: |n_a| <= ceil(rc / width_a) + 1,
    width_a = V / |a_b x a_c| being the cell thickness along a*_a."""
    V = abs(np.linalg.det(cell))
    w = np.array([V / np.linalg.norm(np.cross(cell[(a + 1) % 3], cell[(a + 2) % 3]))
                  for a in range(3)])
    return np.ceil(rc / w).astype(int) + 1


def pair_list_bruteforce(pos: torch.Tensor, cell: np.ndarray, rc: float, targets=None,
                         chunk: int = 4_000_000):
    """All directed pairs (i, j, n) with |R_j + n - R_i| < rc, except i = j, n = 0.

    Plain enumeration over lattice images inside a box of integer vectors.
    Returns (i, j, r) with r = R_j + n - R_i.
    """
    N = pos.shape[0]
    cellt = torch.as_tensor(cell, dtype=torch.float64)
    frac = pos @ torch.linalg.inv(cellt)
    wrapped = (frac - torch.floor(frac)) @ cellt
    nmax = image_range(cell, rc)
    ns = torch.tensor([(a, b, c) for a in range(-nmax[0], nmax[0] + 1)
                       for b in range(-nmax[1], nmax[1] + 1)
                       for c in range(-nmax[2], nmax[2] + 1)], dtype=torch.float64)
    shifts = ns @ cellt
    # Shift between the wrapped and the original positions (keeps r exact in terms of pos).
    off = wrapped - pos
    if targets is None:
        targets = torch.arange(N)
    targets = torch.as_tensor(targets)
    out_i, out_j, out_r = [], [], []
    per = max(1, chunk // max(1, N * len(ns)))
    rc2 = rc * rc
    for t0 in range(0, len(targets), per):
        ti = targets[t0:t0 + per]
        base = (wrapped[None, :, :] - wrapped[ti][:, None, :])      # (T, N, 3)
        r = base[:, :, None, :] + shifts[None, None, :, :]          # (T, N, S, 3)
        r2 = (r * r).sum(-1)
        mask = r2 < rc2
        is_self = (ti[:, None] == torch.arange(N)[None, :])[:, :, None] & \
            (ns.abs().sum(-1) == 0)[None, None, :]
        mask &= ~is_self
        idx = mask.nonzero()
        ii = ti[idx[:, 0]]
        jj = idx[:, 1]
        # Re-express in terms of the original positions so gradients flow.
        rr = pos[jj] - pos[ii] + (off[jj] - off[ii]).detach() + shifts[idx[:, 2]]
        out_i.append(ii)
        out_j.append(jj)
        out_r.append(rr)
    return torch.cat(out_i), torch.cat(out_j), torch.cat(out_r)


def pair_list(pos: torch.Tensor, cell: np.ndarray, rc: float, targets=None):
    """Directed pair list within rc. Uses a periodic k-d tree for orthorhombic
    cells when rc is below half the shortest edge, else brute-force images."""
    cell = np.asarray(cell, float)
    ortho = np.allclose(cell, np.diag(np.diag(cell)))
    L = np.diag(cell)
    if not ortho or rc >= 0.5 * L.min():
        return pair_list_bruteforce(pos, cell, rc, targets)
    from scipy.spatial import cKDTree
    p = pos.detach().numpy()
    w = p - np.floor(p / L) * L
    tree = cKDTree(w, boxsize=L)
    if targets is None:
        pr = tree.query_pairs(rc, output_type="ndarray")
        i = np.concatenate([pr[:, 0], pr[:, 1]])
        j = np.concatenate([pr[:, 1], pr[:, 0]])
    else:
        targets = np.asarray(targets)
        lists = tree.query_ball_point(w[targets], rc)
        i = np.concatenate([np.full(len(l), t) for t, l in zip(targets, lists)]).astype(np.int64)
        j = np.concatenate([np.asarray(l, np.int64) for l in lists])
        keep = i != j
        i, j = i[keep], j[keep]
    i = torch.from_numpy(i.astype(np.int64))
    j = torch.from_numpy(j.astype(np.int64))
    d = (w[j] - w[i])
    shift = -L * np.round(d / L) + (w[j] - p[j]) - (w[i] - p[i])
    r = pos[j] - pos[i] + torch.from_numpy(shift)
    keep = (r * r).sum(-1) < rc * rc
    return i[keep], j[keep], r[keep]


def field_from_pairs(N, i, j, r, radial, dsrc):
    """E_i = sum over pairs (i, j, r) of T(r) d_j for radial (A, B) evaluated at |r|."""
    rn = torch.sqrt((r * r).sum(-1))
    A, B = radial(rn, i, j)
    contrib = apply_pairs(A, B, r, dsrc[j])
    out = torch.zeros((N,) + dsrc.shape[1:], dtype=dsrc.dtype)
    return out.index_add(0, i, contrib)
