"""Stochastic Lanczos quadrature of Tr sqrt(C) (oracle).

Review of SL-MBD section and Algorithms 1-2:
- Hutchinson: Tr sqrt(C) ~ (D/R) sum_l v_l^T sqrt(C) v_l with normalized
  Rademacher probes (eqs. hutch, dds), D = 3N.
- Gauss quadrature: v^T sqrt(C) v ~ sum_k tau_k sqrt(theta_k), nodes theta_k
  the eigenvalues of the tridiagonal Delta = Y^T C Y and weights the squared
  first components of its eigenvectors (eqs. sl3, sl4, tridiag1, tridiag2).
- Lanczos recurrence (eqs. recurs, recurs2): y_1 = v, l_k = C y_k,
  a_k = y_k . l_k, b_{k+1} y_{k+1} = l_k - a_k y_k - b_k y_{k-1},
  b_{k+1} = ||.||.
- Energy: E = 1/2 Tr sqrt(C) - 3/2 sum omega (eq. plasmonic2).

Here "m steps" is the number of matvecs, i.e. the size of Delta (the paper's
M + 1). The oracle re-orthogonalizes every new vector against all earlier
ones with classical Gram-Schmidt applied twice; in exact arithmetic this
changes nothing. A breakdown b_{k+1} <= 1e-12 max(|a_k|, b_k) truncates
Delta at k.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, List

import torch

from .probes import rademacher


@dataclass
class LanczosResult:
    a: torch.Tensor          # (m_eff,)
    b: torch.Tensor          # (m_eff - 1,) off-diagonal b_2..b_m
    Y: torch.Tensor          # (m_eff, D) Krylov basis


def lanczos(matvec: Callable, v: torch.Tensor, m: int, reorth: str = "full",
            breakdown: float = 1e-12) -> LanczosResult:
    """Run m steps from the unit vector v (any shape; flattened internally)."""
    shape = v.shape
    y = v.reshape(-1)
    Y: List[torch.Tensor] = [y]
    a_list, b_list = [], []
    b_prev = None
    for k in range(m):
        l = matvec(Y[k].reshape(shape)).reshape(-1)
        a = torch.dot(Y[k], l)
        a_list.append(a)
        if k == m - 1:
            break
        w = l - a * Y[k]
        if k > 0:
            w = w - b_prev * Y[k - 1]
        if reorth == "full":
            Ym = torch.stack(Y)
            for _ in range(2):
                w = w - Ym.T @ (Ym @ w)
        bn = torch.linalg.norm(w)
        scale = max(abs(float(a.detach())),
                    float(b_prev.detach()) if b_prev is not None else 0.0)
        if float(bn.detach()) <= breakdown * scale:
            break
        b_list.append(bn)
        b_prev = bn
        Y.append(w / bn)
    a_t = torch.stack(a_list)
    b_t = torch.stack(b_list) if b_list else torch.zeros(0, dtype=a_t.dtype)
    return LanczosResult(a_t, b_t[: len(a_list) - 1], torch.stack(Y[: len(a_list)]))


def tridiagonal(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    T = torch.diag(a)
    if b.numel():
        T = T + torch.diag(b, 1) + torch.diag(b, -1)
    return T


def quadrature(a: torch.Tensor, b: torch.Tensor, f=torch.sqrt):
    """sum_k U_1k^2 f(theta_k) for the tridiagonal (a, b); also (theta, weights)."""
    theta, U = torch.linalg.eigh(tridiagonal(a, b))
    wts = U[0, :] ** 2
    return (wts * f(theta)).sum(), theta, wts


@dataclass
class SLQResult:
    energy: torch.Tensor
    trace: torch.Tensor
    q: torch.Tensor              # per-probe quadrature values Q_l
    a: List[torch.Tensor]
    b: List[torch.Tensor]
    theta_min: float


def slq(op: Callable, n_atoms: int, omega, seed: int, n_probes: int, m: int,
        system: int = 0, reorth: str = "full", probes=None) -> SLQResult:
    """E_MBD by stochastic Lanczos quadrature with the shared probe definition."""
    D = 3 * n_atoms
    if probes is None:
        probes = range(n_probes)
    probes = list(probes)
    V = rademacher(seed, system, n_atoms, probes)
    qs, As, Bs = [], [], []
    tmin = float("inf")
    for l in range(len(probes)):
        res = lanczos(op, V[l], m, reorth=reorth)
        q, theta, _ = quadrature(res.a, res.b)
        tmin = min(tmin, float(theta.detach().min()))
        qs.append(q)
        As.append(res.a)
        Bs.append(res.b)
    qv = torch.stack(qs)
    omega = torch.as_tensor(omega, dtype=torch.float64)
    trace = D / len(probes) * qv.sum()
    energy = 0.5 * trace - 1.5 * omega.sum()
    return SLQResult(energy, trace, qv, As, Bs, tmin)
