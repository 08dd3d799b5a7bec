"""Smooth particle-mesh Ewald reciprocal field for dipoles (oracle).

Steps in the paper's order (Theory section, eqs. scaledfractional, spme,
dipolarr; the influence function is the Essmann et al. / Sagui et al. pair
potential that the paper cites):

1. scaled fractional coordinates u_{a j} = K_a a*_a . R_j;
2. cardinal B-splines M_p of order p (support p points, degree p - 1)
   interpolate exp(2 pi i m_a u_a / K_a) ~ b_a(m_a) sum_k M_p(u_a - k) exp(2 pi i m_a k / K_a);
3. the dipole grid D(k) = sum_j d_j . grad_j W_j(k), W_j(k) = prod_a M_p(u_{a j} - k_a)
   with k wrapped periodically;
4. convolution with the influence function G(m) = exp(-pi^2 |m|^2 / tau^2) B(m) / (pi V |m|^2),
   G(0) = 0, B(m) = prod_a |b_a(m_a)|^2, done by FFT;
5. the field is the derivative gather E_i = sum_k grad_i W_i(k) phi(k).

With F+[D](m) = sum_k D(k) e^{+2 pi i m.k/K}, the reciprocal energy is
U = 1/2 sum_m G(m) |F+[D](m)|^2 and phi(k) = sum_m G(m) F+[D](m) e^{-2 pi i m.k/K},
so the field is dU/dd_i. Stencil convention: for u with floor(u) = u0 and
w = u - u0, the p points are k = u0 - t (t = 0..p-1) with weight M_p(w + t).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .exact import recip_vectors


def bspline(p: int, x: torch.Tensor) -> torch.Tensor:
    """Cardinal B-spline M_p(x): M_2(x) = 1 - |x - 1| on [0, 2], and
    M_n(x) = [x M_{n-1}(x) + (n - x) M_{n-1}(x - 1)] / (n - 1)."""
    if p == 2:
        return torch.clamp(1.0 - torch.abs(x - 1.0), min=0.0)
    return (x * bspline(p - 1, x) + (p - x) * bspline(p - 1, x - 1.0)) / (p - 1)


def bspline_deriv(p: int, x: torch.Tensor) -> torch.Tensor:
    """M_p'(x) = M_{p-1}(x) - M_{p-1}(x - 1)."""
    return bspline(p - 1, x) - bspline(p - 1, x - 1.0)


def bmod2(p: int, K: int) -> torch.Tensor:
    """|b(m)|^2 = 1 / |sum_{k=0}^{p-2} M_p(k+1) e^{2 pi i m k / K}|^2 for m = 0..K-1."""
    k = torch.arange(p - 1, dtype=torch.float64)
    Mk = bspline(p, k + 1.0)
    m = torch.arange(K, dtype=torch.float64)
    ph = 2.0 * math.pi * m[:, None] * k[None, :] / K
    re = (Mk[None, :] * torch.cos(ph)).sum(1)
    im = (Mk[None, :] * torch.sin(ph)).sum(1)
    return 1.0 / (re * re + im * im)


def influence(cell, K, p, tau) -> torch.Tensor:
    """G(m) on the full K1 x K2 x K3 grid of DFT indices."""
    cell = np.asarray(cell, float)
    V = abs(float(np.linalg.det(cell)))
    rec = torch.from_numpy(recip_vectors(cell))
    axes = []
    for a in range(3):
        m = torch.arange(K[a], dtype=torch.float64)
        axes.append(torch.where(m <= K[a] // 2, m, m - K[a]))
    g1, g2, g3 = torch.meshgrid(*axes, indexing="ij")
    mv = g1[..., None] * rec[0] + g2[..., None] * rec[1] + g3[..., None] * rec[2]
    mm = (mv * mv).sum(-1)
    Bm = bmod2(p, K[0])[:, None, None] * bmod2(p, K[1])[None, :, None] * \
        bmod2(p, K[2])[None, None, :]
    safe = torch.where(mm > 0, mm, torch.ones_like(mm))
    G = torch.exp(-math.pi ** 2 * mm / tau ** 2) * Bm / (math.pi * V * safe)
    return torch.where(mm > 0, G, torch.zeros_like(G))


def _stencil(pos, cell, K, p):
    """Base indices, per-axis weights M_p(w + t) and derivatives for t = 0..p-1."""
    rec = torch.from_numpy(recip_vectors(cell))
    Kt = torch.tensor(K, dtype=torch.float64)
    u = (pos @ rec.T) * Kt[None, :]                   # (N, 3)
    u0 = torch.floor(u.detach())
    w = u - u0
    t = torch.arange(p, dtype=torch.float64)
    x = w[:, :, None] + t[None, None, :]              # (N, 3, p)
    return u0.long(), bspline(p, x), bspline_deriv(p, x), rec, Kt


def spread(pos, cell, K, p, dvec):
    """Dipole grid D(k) from dipoles dvec (N, 3, B); returns (K1, K2, K3, B)."""
    N = pos.shape[0]
    u0, M, dM, rec, Kt = _stencil(pos, cell, K, p)
    # Dipole in scaled fractional coordinates: dd_a = K_a a*_a . d.
    dd = torch.einsum("ac,ncb->nab", rec * Kt[:, None], dvec)      # (N, 3, B)
    B = dvec.shape[2]
    grid = torch.zeros(K[0] * K[1] * K[2], B, dtype=torch.float64)
    for t1 in range(p):
        i1 = (u0[:, 0] - t1) % K[0]
        for t2 in range(p):
            i2 = (u0[:, 1] - t2) % K[1]
            for t3 in range(p):
                i3 = (u0[:, 2] - t3) % K[2]
                c = (dd[:, 0, :] * (dM[:, 0, t1] * M[:, 1, t2] * M[:, 2, t3])[:, None]
                     + dd[:, 1, :] * (M[:, 0, t1] * dM[:, 1, t2] * M[:, 2, t3])[:, None]
                     + dd[:, 2, :] * (M[:, 0, t1] * M[:, 1, t2] * dM[:, 2, t3])[:, None])
                flat = (i1 * K[1] + i2) * K[2] + i3
                grid = grid.index_add(0, flat, c)
    return grid.reshape(K[0], K[1], K[2], B)


def convolve(grid, G):
    """phi = sum_m G(m) F+[D](m) e^{-2 pi i m.k/K} with unnormalized transforms."""
    Kprod = grid.shape[0] * grid.shape[1] * grid.shape[2]
    Fp = torch.fft.ifftn(grid, dim=(0, 1, 2)) * Kprod
    return torch.fft.fftn(G[..., None] * Fp, dim=(0, 1, 2)).real


def gather(pos, cell, K, p, phi):
    """E_i = sum_k grad_i W_i(k) phi(k) for phi (K1, K2, K3, B); returns (N, 3, B)."""
    u0, M, dM, rec, Kt = _stencil(pos, cell, K, p)
    N = pos.shape[0]
    B = phi.shape[3]
    flatphi = phi.reshape(-1, B)
    gfrac = torch.zeros(N, 3, B, dtype=torch.float64)
    for t1 in range(p):
        i1 = (u0[:, 0] - t1) % K[0]
        for t2 in range(p):
            i2 = (u0[:, 1] - t2) % K[1]
            for t3 in range(p):
                i3 = (u0[:, 2] - t3) % K[2]
                v = flatphi[(i1 * K[1] + i2) * K[2] + i3]           # (N, B)
                gfrac = gfrac + torch.stack([
                    (dM[:, 0, t1] * M[:, 1, t2] * M[:, 2, t3])[:, None] * v,
                    (M[:, 0, t1] * dM[:, 1, t2] * M[:, 2, t3])[:, None] * v,
                    (M[:, 0, t1] * M[:, 1, t2] * dM[:, 2, t3])[:, None] * v], dim=1)
    # Cartesian gradient: d/dR = sum_a K_a a*_a d/du_a.
    return torch.einsum("ac,nab->ncb", rec * Kt[:, None], gfrac)


def recip_field(pos, cell, K, p, tau, dvec):
    """SPME approximation of (T_rec d) at every atom; dvec (N, 3, B)."""
    G = influence(cell, K, p, tau)
    return gather(pos, cell, K, p, convolve(spread(pos, cell, K, p, dvec), G))
