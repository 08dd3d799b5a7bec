"""Block Lanczos quadrature on the GPU (krylov_block > 1) against the oracle's block
recurrence with the same probes and the same SPME operator.

Tolerances as for the single-probe path: float64 1e-9 relative on the energy and 1e-8
on each probe's value (rounding through m block steps and two Cholesky-QR passes per
step); mixed precision 1e-5 on the energy and 1e-4 on each probe's value."""
import numpy as np
import pytest
import torch

import synth
from oracle import block_lanczos as obl
from oracle import method as om

pytestmark = pytest.mark.gpu

A = synth.ANGSTROM_BOHR
SEED = 12345


def _plan(s, prec, kb, R, m, block, graph=False, reorth=0):
    import paper_2307_02278_amd as P
    ds = P.DeviceSystem(s.pos, s.cell, s.alpha, s.omega, s.rvdw)
    prm = P.Params(ewald_tau=0.35 * synth.BOHR_ANGSTROM, real_cutoff=13.0 * A, grid=(16, 16, 16),
                   n_probes=R, n_steps=m, block=block, precision=prec, seed=SEED,
                   krylov_block=kb, graph=graph, reorth=reorth)
    return P.Plan([ds], prm)


def _oracle(s, plan, R, m, kb):
    inf = plan.info(0)
    op = om.Operator(s, om.MethodParams(tau=inf.tau, r_pair=inf.r_pair, grid=tuple(inf.grid),
                                        order=inf.spline_order))
    return obl.block_slq(op, s.n, s.omega, seed=SEED, n_probes=R, m=m, b=kb)


@pytest.fixture(scope="module")
def tiny():
    return synth.workload("tiny").systems[0]


@pytest.mark.parametrize("kb,block", [(2, 16), (4, 16), (8, 16), (4, 64)])
def test_block_fp64_matches_oracle(tiny, kb, block):
    import paper_2307_02278_amd as P
    R, m = 16, 10
    plan = _plan(tiny, P.PREC_FP64, kb, R, m, block)
    e = float(plan.execute()[0])
    plan.check()
    q = plan.quadrature()
    e_ref, q_ref = _oracle(tiny, plan, R, m, kb)
    assert e == pytest.approx(float(e_ref), rel=1e-9)
    assert torch.allclose(q, q_ref, rtol=1e-8, atol=0)


def test_block_mixed_matches_oracle(tiny):
    import paper_2307_02278_amd as P
    R, m, kb = 16, 10, 4
    plan = _plan(tiny, P.PREC_MIXED, kb, R, m, 16)
    e = float(plan.execute()[0])
    plan.check()
    e_ref, q_ref = _oracle(tiny, plan, R, m, kb)
    assert e == pytest.approx(float(e_ref), rel=1e-5)
    assert torch.allclose(plan.quadrature(), q_ref, rtol=1e-4, atol=0)


def test_block_ragged_batches(tiny):
    """R = 24 probes with B = 16: one full batch and one of 8 probes (two live Krylov
    blocks of 4, two empty ones)."""
    import paper_2307_02278_amd as P
    R, m, kb = 24, 8, 4
    plan = _plan(tiny, P.PREC_FP64, kb, R, m, 16)
    e = float(plan.execute()[0])
    plan.check()
    e_ref, q_ref = _oracle(tiny, plan, R, m, kb)
    assert e == pytest.approx(float(e_ref), rel=1e-9)
    assert torch.allclose(plan.quadrature(), q_ref, rtol=1e-8, atol=0)


def test_block_exhausted_krylov_space():
    """Four atoms: D = 12 = m kb, the block rule is exact for the operator; a longer run
    ends the block on its rank-deficient residual and gives the same values."""
    import paper_2307_02278_amd as P
    s = synth.tiny_random(seed=4, n=4, L_ang=6.0, dmin_ang=2.2)
    R, kb = 4, 4
    exact = _plan(s, P.PREC_FP64, kb, R, 3, 4)
    e3 = float(exact.execute()[0])
    exact.check()
    e_ref, q_ref = _oracle(s, exact, R, 3, kb)
    assert e3 == pytest.approx(float(e_ref), rel=1e-9)
    longer = _plan(s, P.PREC_FP64, kb, R, 6, 4)
    e6 = float(longer.execute()[0])
    longer.check()
    assert e6 == pytest.approx(e3, rel=1e-8)


def test_block_graph_replay_matches_eager(tiny):
    import paper_2307_02278_amd as P
    eager = _plan(tiny, P.PREC_MIXED, 4, 16, 8, 16)
    graph = _plan(tiny, P.PREC_MIXED, 4, 16, 8, 16, graph=True)
    ref = eager.execute().clone()
    eager.check()
    for rep in range(3):
        e = graph.execute()
        graph.check()
        assert torch.equal(e, ref), rep
        _ = eager.execute()
        torch.cuda.synchronize()


def test_block_plan_has_no_scalar_tridiagonal(tiny):
    import paper_2307_02278_amd as P
    plan = _plan(tiny, P.PREC_FP64, 2, 4, 4, 4)
    plan.execute()
    plan.check()
    with pytest.raises(P.MbdError) as ei:
        plan.tridiagonal()
    assert ei.value.code == P.MBD_E_STATE
