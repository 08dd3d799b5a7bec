"""Pins of the oracle's block Lanczos quadrature.

- b = 1 is the ordinary Lanczos rule: the block oracle equals the (separately pinned)
  single-probe oracle without re-orthogonalization, probe by probe;
- block Gauss exactness: after m block steps R_0^T E_1^T T^j E_1 R_0 = V^T C^j V for
  every j <= 2m - 1 (a random SPD matrix, computed by plain matrix powers);
- a Krylov space exhausted exactly (m b = D) makes the rule exact: it equals
  V^T sqrt(C) V from the eigendecomposition of C;
- a rank-deficient residual block stops the recurrence with finite values.
"""
import pytest
import torch

import synth
from oracle import block_lanczos as obl
from oracle import lanczos as olz
from oracle import method as om
from oracle.probes import rademacher


def _spd(D, seed, lo=0.2, hi=3.0):
    g = torch.Generator().manual_seed(seed)
    Q, _ = torch.linalg.qr(torch.randn(D, D, dtype=torch.float64, generator=g))
    ev = lo + (hi - lo) * torch.rand(D, dtype=torch.float64, generator=g)
    return Q @ torch.diag(ev) @ Q.T


def test_block_size_one_is_the_lanczos_rule():
    s = synth.tiny_random(seed=2, n=30, L_ang=8.0)
    A = synth.ANGSTROM_BOHR
    op = om.Operator(s, om.MethodParams(tau=0.2, r_pair=13.0 * A, grid=(16, 16, 16)))
    e1, q1 = obl.block_slq(op, s.n, s.omega, seed=7, n_probes=3, m=8, b=1)
    ref = olz.slq(op, s.n, s.omega, seed=7, n_probes=3, m=8, reorth="none")
    assert torch.allclose(q1, ref.q, rtol=1e-12, atol=0)
    assert float(e1) == pytest.approx(float(ref.energy), rel=1e-12)


@pytest.mark.parametrize("D,b,m", [(60, 3, 4), (48, 4, 3), (40, 2, 6)])
def test_block_gauss_rule_matches_moments(D, b, m):
    C = _spd(D, seed=D + b)
    V = torch.randn(D, b, dtype=torch.float64, generator=torch.Generator().manual_seed(3))
    As, Bs, R0 = obl.block_lanczos(lambda Y: C @ Y, V, m)
    assert len(As) == m
    T = obl.block_tridiagonal(As, Bs)
    E1 = torch.zeros(m * b, b, dtype=torch.float64)
    E1[:b] = torch.eye(b, dtype=torch.float64)
    Tj = torch.eye(m * b, dtype=torch.float64)
    Cj = torch.eye(D, dtype=torch.float64)
    for j in range(2 * m):
        lhs = R0.T @ E1.T @ Tj @ E1 @ R0
        rhs = V.T @ Cj @ V
        assert torch.allclose(lhs, rhs, rtol=1e-9, atol=1e-9 * float(rhs.abs().max())), j
        Tj = Tj @ T
        Cj = Cj @ C


def test_exhausted_krylov_space_is_exact():
    D, b = 12, 4
    C = _spd(D, seed=5)
    V = rademacher(3, 0, D // 3, range(b)).reshape(b, D).T
    As, Bs, R0 = obl.block_lanczos(lambda Y: C @ Y, V, D // b)
    got = obl.block_quadrature(As, Bs, R0)
    th, U = torch.linalg.eigh(C)
    want = V.T @ U @ torch.diag(torch.sqrt(th)) @ U.T @ V
    assert torch.allclose(got, want, rtol=1e-10, atol=1e-12)


def test_exhausted_space_stops_and_stays_exact():
    D, b = 12, 4
    C = _spd(D, seed=5)
    V = rademacher(3, 0, D // 3, range(b)).reshape(b, D).T
    As, Bs, R0 = obl.block_lanczos(lambda Y: C @ Y, V, 6)
    assert len(As) == D // b
    th, U = torch.linalg.eigh(C)
    want = V.T @ U @ torch.diag(torch.sqrt(th)) @ U.T @ V
    assert torch.allclose(obl.block_quadrature(As, Bs, R0), want, rtol=1e-10, atol=1e-12)


def test_rank_deficient_residual_stops_the_block():
    D, b = 6, 4
    C = _spd(D, seed=9)
    V = torch.randn(D, b, dtype=torch.float64, generator=torch.Generator().manual_seed(1))
    As, Bs, R0 = obl.block_lanczos(lambda Y: C @ Y, V, 5)
    assert len(As) == 1 and len(Bs) == 0
    q = obl.block_quadrature(As, Bs, R0)
    assert torch.isfinite(q).all()
