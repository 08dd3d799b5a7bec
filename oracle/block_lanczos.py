"""Block stochastic Lanczos quadrature of Tr sqrt(C) (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The Conclusions name the parallel structure of the estimator (independent probes plus
one reduction); the block form runs the Lanczos recurrence of Algorithm 2 on blocks
of b probes at once, so that every step multiplies C into a b-column block and the
Krylov space of the block is b times wider for the same number of steps. With the
probe block V (D x b) and its QR factorization V = Y_1 R_0:

  C Y_k = Y_{k-1} B_{k-1}^T + Y_k A_k + Y_{k+1} B_k,
  A_k = Y_k^T C Y_k,   Y_{k+1} B_k = C Y_k - Y_k A_k - Y_{k-1} B_{k-1}^T (QR),

and the block tridiagonal T (m b x m b) with diagonal blocks A_k and sub-diagonal
blocks B_k gives the block Gauss rule

  V^T f(C) V ~ R_0^T E_1^T f(T) E_1 R_0,   E_1 = the first b columns of I.

Per probe l, Q_l is the l-th diagonal entry of that b x b matrix; the energy is
E = 1/2 (D / R) sum_l Q_l - 3/2 sum omega as for single probes (b = 1 reduces to the
ordinary Lanczos rule). A block whose new residual block is numerically rank
deficient stops there and T keeps the steps done: a Cholesky pivot of W^T W below
(1e-10 s)^2, with s = max_i (A_k)_ii the scale of the step (for the probe block, s^2 =
the largest diagonal entry of V^T V). No re-orthogonalization (the plain recurrence).
"""
from __future__ import annotations

from typing import Callable, List

import torch

from .probes import rademacher

BREAKDOWN = 1e-10


def _qr(W: torch.Tensor, scale=None):
    """W = Y R with R upper triangular with a positive diagonal (Cholesky of W^T W,
    twice); None if W^T W is numerically singular against the scale."""
    Y, R = W, torch.eye(W.shape[1], dtype=W.dtype)
    for p in range(2):
        G = Y.T @ Y
        s2 = float(torch.diagonal(G).max()) if (scale is None or p == 1) else scale * scale
        L, info = torch.linalg.cholesky_ex(G)
        if int(info) != 0 or float(torch.diagonal(L).min() ** 2) <= BREAKDOWN ** 2 * s2:
            return None
        Rk = L.T
        Y = torch.linalg.solve_triangular(Rk, Y, upper=True, left=False)
        R = Rk @ R
    return Y, R


def block_lanczos(matvec: Callable, V: torch.Tensor, m: int):
    """m block steps from the probe block V (D x b). Returns (A list, B list, R0)."""
    q0 = _qr(V)
    if q0 is None:
        raise ValueError("probe block is rank deficient")
    Y, R0 = q0
    Ys: List[torch.Tensor] = [Y]
    As, Bs = [], []
    for k in range(m):
        L = matvec(Ys[k])
        A = Ys[k].T @ L
        As.append(0.5 * (A + A.T))
        if k == m - 1:
            break
        W = L - Ys[k] @ As[k]
        if k > 0:
            W = W - Ys[k - 1] @ Bs[k - 1].T
        q = _qr(W, scale=float(torch.diagonal(As[k]).max()))
        if q is None:
            break
        Ys.append(q[0])
        Bs.append(q[1])
    return As, Bs[: len(As) - 1], R0


def block_tridiagonal(As, Bs) -> torch.Tensor:
    b = As[0].shape[0]
    n = len(As) * b
    T = torch.zeros(n, n, dtype=As[0].dtype)
    for k, A in enumerate(As):
        T[k * b:(k + 1) * b, k * b:(k + 1) * b] = A
    for k, Bk in enumerate(Bs):
        T[(k + 1) * b:(k + 2) * b, k * b:(k + 1) * b] = Bk
        T[k * b:(k + 1) * b, (k + 1) * b:(k + 2) * b] = Bk.T
    return T


def block_quadrature(As, Bs, R0, f=torch.sqrt) -> torch.Tensor:
    """R_0^T E_1^T f(T) E_1 R_0 (b x b)."""
    b = R0.shape[0]
    theta, U = torch.linalg.eigh(block_tridiagonal(As, Bs))
    P = U[:b, :]                       # E_1^T U
    M = P @ torch.diag(f(theta)) @ P.T
    return R0.T @ M @ R0


def block_slq(op: Callable, n_atoms: int, omega, seed: int, n_probes: int, m: int, b: int,
              system: int = 0):
    """E_MBD by block SLQ: probes 0..R-1 in consecutive blocks of b (R divisible by b).
    Returns (energy, per-probe Q)."""
    if n_probes % b:
        raise ValueError("n_probes must be a multiple of the block size")
    D = 3 * n_atoms
    V = rademacher(seed, system, n_atoms, range(n_probes))     # (R, N, 3)

    def mv(Y):  # (D, b) -> (D, b) through the operator's (N, 3, b) layout
        out = op(Y.T.reshape(-1, n_atoms, 3).permute(1, 2, 0))
        return out.permute(2, 0, 1).reshape(Y.shape[1], D).T

    qs = []
    for l0 in range(0, n_probes, b):
        Vb = V[l0:l0 + b].reshape(b, D).T
        As, Bs, R0 = block_lanczos(mv, Vb, m)
        qs.append(torch.diagonal(block_quadrature(As, Bs, R0)))
    q = torch.cat(qs)
    omega = torch.as_tensor(omega, dtype=torch.float64)
    energy = 0.5 * D / n_probes * q.sum() - 1.5 * omega.sum()
    return energy, q
