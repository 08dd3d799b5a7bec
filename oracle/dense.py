"""Exact MBD energy from the full spectrum (oracle).

E_MBD = 1/2 sum_i sqrt(lambda_i(C)) - 3/2 sum_i omega_i (eq. plasmonic), which
equals 1/2 Tr sqrt(C) - 3/2 sum omega (eq. plasmonic2). C must be positive
definite. Forces are F = -dE/dR; the analytic eigen-gradient
dE/dR = 1/4 Tr(C^{-1/2} dC/dR) is what automatic differentiation of this
function through a symmetric eigensolver returns.
"""
from __future__ import annotations

import torch


def energy_from_C(C: torch.Tensor, omega) -> torch.Tensor:
    lam = torch.linalg.eigvalsh(C)
    if float(lam.detach().min()) <= 0.0:
        raise ValueError(f"C is not positive definite (lambda_min = {float(lam.detach().min()):.3e})")
    omega = torch.as_tensor(omega, dtype=torch.float64)
    return 0.5 * torch.sqrt(lam).sum() - 1.5 * omega.sum()


def sqrt_trace_probe(C: torch.Tensor, v: torch.Tensor) -> torch.Tensor:
    """v^T sqrt(C) v through the eigendecomposition (eq. sl1)."""
    lam, W = torch.linalg.eigh(C)
    mu = W.T @ v.reshape(-1)
    return (mu * mu * torch.sqrt(lam)).sum()
