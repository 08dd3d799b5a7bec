"""The SPME-Lanczos matvec (oracle): l = Omega y + Diag(g) E*(g * y).

Theory section: C = Omega + V~ (eq. ccd) with g = (+)_i omega_i sqrt(alpha_i) 1_3
(eq. gvec); the generalized dipoles d = g * y (Hadamard product) produce the
generalized field E* = E_dir + E_rec + E_self (eq. ewalddip), and
l = Omega y + Diag(g) E* (eq. lk3).

- E_dir: pairs within the direct-space cutoff r_pair over all images, kernel
  T_erfc - (1 - f) T (eq. fld_ewald, computed with a neighbour list);
- E_rec: smooth PME (eq. spme) with grid K, spline order p;
- E_self: -(4 tau^3 / (3 sqrt(pi))) d (eq. fld_ewald1, energy-convention
  field coefficient).

The cutoff r_pair, tau, K and p are parameters of the method; the oracle's
exact module gives the limit they approximate.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Sequence

import torch

from . import spme as sp
from . import tensors as tz
from .exact import self_coefficient

DIAG, DIR, REC, SELF, ALL = 1, 2, 4, 8, 15


@dataclass
class MethodParams:
    tau: float                 # bohr^-1
    r_pair: float              # bohr
    grid: Sequence[int]        # (K1, K2, K3)
    order: int = 6
    beta: float = 0.83
    d: float = 6.0


class Operator:
    """C applied matrix-free to blocks y of shape (N, 3, B).

    The pair list and spline stencils depend only on positions; they are
    rebuilt on every call so that automatic differentiation with respect to
    positions sees the whole dependence.
    """

    def __init__(self, sys, mp: MethodParams, pos=None):
        self.sys = sys
        self.mp = mp
        self.pos = torch.as_tensor(sys.pos if pos is None else pos, dtype=torch.float64)
        self.alpha = torch.as_tensor(sys.alpha, dtype=torch.float64)
        self.omega = torch.as_tensor(sys.omega, dtype=torch.float64)
        self.rvdw = torch.as_tensor(sys.rvdw, dtype=torch.float64)
        self.g = self.omega * torch.sqrt(self.alpha)
        self.G = sp.influence(sys.cell, list(mp.grid), mp.order, mp.tau)
        pd = self.pos.detach()
        i, j, _ = tz.pair_list(pd, sys.cell, mp.r_pair)
        self._pairs = (i, j, _ - (pd[j] - pd[i]))     # keep the integer image shift

    def pairs(self):
        i, j, shift = self._pairs
        return i, j, self.pos[j] - self.pos[i] + shift

    def field(self, d, components=ALL):
        """E* for dipoles d (N, 3, B), selected parts."""
        N = self.pos.shape[0]
        E = torch.zeros_like(d)
        if components & DIR:
            i, j, r = self.pairs()
            rn = torch.sqrt((r * r).sum(-1))
            A, B = tz.radial_direct(rn, self.mp.tau,
                                    self.mp.beta * (self.rvdw[i] + self.rvdw[j]), self.mp.d)
            E = E.index_add(0, i, tz.apply_pairs(A, B, r, d[j]))
        if components & REC:
            grid = sp.spread(self.pos, self.sys.cell, list(self.mp.grid), self.mp.order, d)
            phi = sp.convolve(grid, self.G)
            E = E + sp.gather(self.pos, self.sys.cell, list(self.mp.grid), self.mp.order, phi)
        if components & SELF:
            E = E + self_coefficient(self.mp.tau) * d
        return E

    def __call__(self, y, components=ALL):
        squeeze = y.dim() == 2
        y = y[..., None] if squeeze else y
        g = self.g[:, None, None]
        out = g * self.field(g * y, components)
        if components & DIAG:
            out = out + (self.omega ** 2)[:, None, None] * y
        return out[..., 0] if squeeze else out
