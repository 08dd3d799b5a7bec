"""Converged Ewald summation of the periodic damped dipole tensor (oracle).

Definition (energy convention, tin-foil boundary, m = 0 omitted as in
eq. fld_ewald2):

  T^pbc_ij = sum'_n T_dir(r_ij + n) + T_rec(r_ij) + delta_ij T_self
  T_dir    = T_erfc - (1 - f_ij) T                  (eq. fld_ewald)
  T_rec(r) = (4 pi / V) sum_{m != 0} exp(-pi^2 m^2 / tau^2) (m m^T / m^2) cos(2 pi m.r)
  T_self   = -(4 tau^3 / (3 sqrt(pi))) I

The primed sum excludes i = j with n = 0 and includes every other image, also
i = j with n != 0. r_ij = R_j - R_i. The reciprocal sum is the dipolar form of
eq. fld_ewald2 with the structure factor of eq. structurefactor, written so
that the result is real; the self coefficient is the one that makes T^pbc
independent of tau (the printed 2 tau^3 / (3 sqrt(pi)) is the self-energy
coefficient of a dipole, not of its field).

The coupling matrix (eq. ham) is C = Omega + G T^pbc G with
Omega = diag(omega_i^2 I_3) and G = diag(omega_i sqrt(alpha_i) I_3) (eqs. ccd, gvec).

Convergence: real space to tau r >= 6 for the erfc part and to r >= 7.2 S_max
for the damping correction (1 - f < 1e-16); reciprocal space to
pi |m| / tau >= 6.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import tensors as tz


def recip_vectors(cell: np.ndarray) -> np.ndarray:
    """Rows a*_a with a*_a . a_b = delta_ab."""
    return np.linalg.inv(np.asarray(cell, float)).T


def m_vectors(cell: np.ndarray, tau: float, cut: float = 6.0, half: bool = True):
    """Reciprocal lattice vectors m != 0 with pi |m| / tau <= cut (one of each +-m pair)."""
    rec = recip_vectors(cell)
    mmax = cut * tau / math.pi
    nmax = [int(math.ceil(mmax * np.linalg.norm(np.asarray(cell)[a]))) for a in range(3)]
    ns = np.array([(a, b, c) for a in range(-nmax[0], nmax[0] + 1)
                   for b in range(-nmax[1], nmax[1] + 1)
                   for c in range(-nmax[2], nmax[2] + 1)], float)
    m = ns @ rec
    mm = np.einsum("kc,kc->k", m, m)
    keep = (mm > 0) & (mm <= mmax * mmax)
    if half:
        # Keep the half space: first nonzero integer component positive.
        first = np.where(ns[:, 0] != 0, ns[:, 0], np.where(ns[:, 1] != 0, ns[:, 1], ns[:, 2]))
        keep &= first > 0
    return torch.from_numpy(m[keep]), torch.from_numpy(ns[keep])


def damping_S(rvdw: torch.Tensor, beta: float):
    return beta * (rvdw[:, None] + rvdw[None, :])


def real_space_dense(pos, cell, tau, rvdw, beta, d):
    """sum'_n T_dir(r_ij + n) assembled as a (N, 3, N, 3) array."""
    N = pos.shape[0]
    S = damping_S(rvdw, beta)
    rc = max(6.0 / tau, 7.2 * float(S.max()))
    i, j, r = tz.pair_list_bruteforce(pos, cell, rc)
    rn = torch.sqrt((r * r).sum(-1))
    A, B = tz.radial_direct(rn, tau, S[i, j], d)
    blk = A[:, None, None] * torch.eye(3, dtype=torch.float64) - \
        B[:, None, None] * r[:, :, None] * r[:, None, :]
    T = torch.zeros(N, N, 3, 3, dtype=torch.float64)
    T = T.index_put((i, j), blk, accumulate=True)
    return T.permute(0, 2, 1, 3)


def recip_dense(pos, cell, tau):
    """T_rec(R_j - R_i) for all i, j as (N, 3, N, 3), via X X^T over half-space m."""
    N = pos.shape[0]
    V = abs(float(np.linalg.det(cell)))
    m, _ = m_vectors(cell, tau)
    mm = (m * m).sum(-1)
    w = 2.0 * (4.0 * math.pi / V) * torch.exp(-math.pi ** 2 * mm / tau ** 2) / mm
    ph = 2.0 * math.pi * (pos @ m.T)                              # (N, K)
    # X[(i,a),(k,cos|sin)] = sqrt(w_k) m_ka {cos, sin}(2 pi m_k . R_i)
    sq = torch.sqrt(w)
    Xc = torch.cos(ph)[:, None, :] * (m.T[None, :, :] * sq[None, None, :])
    Xs = torch.sin(ph)[:, None, :] * (m.T[None, :, :] * sq[None, None, :])
    X = torch.cat([Xc, Xs], dim=2).reshape(3 * N, -1)
    return (X @ X.T).reshape(N, 3, N, 3)


def self_coefficient(tau: float) -> float:
    return -4.0 * tau ** 3 / (3.0 * math.sqrt(math.pi))


def tpbc_dense(pos, cell, tau, rvdw, beta, d):
    """Converged T^pbc as a (3N, 3N) matrix (rows/cols ordered atom-major)."""
    pos = torch.as_tensor(pos, dtype=torch.float64)
    rvdw = torch.as_tensor(rvdw, dtype=torch.float64)
    N = pos.shape[0]
    T = real_space_dense(pos, cell, tau, rvdw, beta, d) + recip_dense(pos, cell, tau)
    T = T.reshape(3 * N, 3 * N)
    return T + self_coefficient(tau) * torch.eye(3 * N, dtype=torch.float64)


def coupling_from_T(T, alpha, omega):
    alpha = torch.as_tensor(alpha, dtype=torch.float64)
    omega = torch.as_tensor(omega, dtype=torch.float64)
    g = (omega * torch.sqrt(alpha)).repeat_interleave(3)
    Om = (omega * omega).repeat_interleave(3)
    return torch.diag(Om) + g[:, None] * T * g[None, :]


def coupling_dense(sys, tau, beta, d, pos=None):
    """Dense C = Omega + G T^pbc G for a synth.System (or explicit positions)."""
    p = torch.as_tensor(sys.pos if pos is None else pos, dtype=torch.float64)
    T = tpbc_dense(p, sys.cell, tau, sys.rvdw, beta, d)
    return coupling_from_T(T, sys.alpha, sys.omega)


def coupling_free(sys, beta, d, pos=None):
    """Free-space (non-periodic) C with the damped tensor f T between distinct atoms."""
    p = torch.as_tensor(sys.pos if pos is None else pos, dtype=torch.float64)
    N = p.shape[0]
    rvdw = torch.as_tensor(sys.rvdw, dtype=torch.float64)
    S = damping_S(rvdw, beta)
    r = p[None, :, :] - p[:, None, :]
    rn = torch.sqrt((r * r).sum(-1) + torch.eye(N, dtype=torch.float64))
    A, B = tz.radial_damped(rn, S, d)
    blk = A[..., None, None] * torch.eye(3, dtype=torch.float64) - \
        B[..., None, None] * r[..., :, None] * r[..., None, :]
    blk = blk * (1.0 - torch.eye(N, dtype=torch.float64))[..., None, None]
    T = blk.permute(0, 2, 1, 3).reshape(3 * N, 3 * N)
    return coupling_from_T(T, sys.alpha, sys.omega)


# ---------------------------------------------------------------------------
# Matrix-free exact field (any N): real space over converged pair lists,
# reciprocal space from dipolar structure factors built with per-axis phases.
# ---------------------------------------------------------------------------

def _structure_factor_field(pos, cell, tau, dvec, targets):
    """(T_rec d) at the target atoms; dvec (N, 3, B)."""
    rec = torch.from_numpy(recip_vectors(cell))
    V = abs(float(np.linalg.det(cell)))
    mmax = 6.0 * tau / math.pi
    nmax = [int(math.ceil(mmax * np.linalg.norm(np.asarray(cell)[a]))) for a in range(3)]
    s = pos @ rec.T                                                # fractional (N, 3)
    dd = torch.einsum("ac,ncb->nab", rec, dvec)                    # a*_a . d_j  (N, 3, B)
    n1 = torch.arange(-nmax[0], nmax[0] + 1, dtype=torch.float64)
    n2 = torch.arange(-nmax[1], nmax[1] + 1, dtype=torch.float64)
    P1 = torch.exp(2j * math.pi * s[:, 0:1] * n1[None, :])        # (N, n1)
    P2 = torch.exp(2j * math.pi * s[:, 1:2] * n2[None, :])
    st = s[targets]
    Q1 = torch.exp(-2j * math.pi * st[:, 0:1] * n1[None, :])
    Q2 = torch.exp(-2j * math.pi * st[:, 1:2] * n2[None, :])
    Bn = dvec.shape[2]
    out = torch.zeros(len(targets), 3, Bn, dtype=torch.float64)
    N1, N2 = len(n1), len(n2)
    g1, g2 = torch.meshgrid(n1, n2, indexing="ij")
    for k3 in range(-nmax[2], nmax[2] + 1):
        P3 = torch.exp(2j * math.pi * s[:, 2] * k3)                # (N,)
        Q3 = torch.exp(-2j * math.pi * st[:, 2] * k3)
        nvec = torch.stack([g1, g2, torch.full_like(g1, float(k3))], -1)   # (N1, N2, 3)
        m = nvec @ rec                                              # (N1, N2, 3)
        mm = (m * m).sum(-1)
        ok = (mm > 0) & (mm <= mmax * mmax)
        if not ok.any():
            continue
        coef = torch.where(ok, (4.0 * math.pi / V) * torch.exp(-math.pi ** 2 * mm / tau ** 2)
                           / torch.where(ok, mm, torch.ones_like(mm)), torch.zeros_like(mm))
        # S(m) = sum_j (m . d_j) e^{2 pi i m . R_j} = sum_a n_a sum_j dd_ja e^{...}
        W = (P2 * P3[:, None])                                      # (N, N2)
        Sa = []
        for a in range(3):
            A = W[:, None, :] * dd[:, a, :, None].to(torch.complex128)   # (N, B, N2)
            Sa.append(torch.einsum("nx,nby->bxy", P1, A))               # (B, N1, N2)
        S = sum(nvec[None, :, :, a] * Sa[a] for a in range(3))           # (B, N1, N2)
        H = coef[None] * S                                               # (B, N1, N2)
        # field_i = sum_m coef m Re[e^{-2 pi i m.R_i} S(m)]  (cos(2 pi m.(R_i-R_j)) form)
        Wt = Q2 * Q3[:, None]                                            # (T, N2)
        for c in range(3):
            mc = m[:, :, c]
            inner_c = torch.einsum("bxy,ty->btx", H * mc[None], Wt)
            val = torch.einsum("btx,tx->tb", inner_c, Q1).real
            out[:, c, :] += val
    return out


def matvec_exact(sys, tau, beta, d, y, targets=None, components=15):
    """Exact (converged Ewald) C y at the target atoms; y (N, 3) or (N, 3, B).

    components: bit mask 1 = Omega y, 2 = direct space, 4 = reciprocal, 8 = self.
    """
    pos = torch.as_tensor(sys.pos, dtype=torch.float64)
    N = pos.shape[0]
    squeeze = y.dim() == 2
    y = y[..., None] if squeeze else y
    alpha = torch.as_tensor(sys.alpha, dtype=torch.float64)
    omega = torch.as_tensor(sys.omega, dtype=torch.float64)
    rvdw = torch.as_tensor(sys.rvdw, dtype=torch.float64)
    g = omega * torch.sqrt(alpha)
    dv = g[:, None, None] * y
    if targets is None:
        targets = torch.arange(N)
    targets = torch.as_tensor(targets)
    E = torch.zeros(len(targets), 3, y.shape[2], dtype=torch.float64)
    if components & 2:
        S_all = beta * 2.0 * float(rvdw.max())
        rc = max(6.0 / tau, 7.2 * S_all)
        i, j, r = tz.pair_list(pos, sys.cell, rc, targets=targets)
        loc = torch.full((N,), -1, dtype=torch.long)
        loc[targets] = torch.arange(len(targets))
        rn = torch.sqrt((r * r).sum(-1))
        A, B = tz.radial_direct(rn, tau, beta * (rvdw[i] + rvdw[j]), d)
        E = E.index_add(0, loc[i], tz.apply_pairs(A, B, r, dv[j]))
    if components & 4:
        E = E + _structure_factor_field(pos, sys.cell, tau, dv, targets)
    if components & 8:
        E = E + self_coefficient(tau) * dv[targets]
    out = g[targets][:, None, None] * E
    if components & 1:
        out = out + (omega[targets] ** 2)[:, None, None] * y[targets]
    return out[..., 0] if squeeze else out
