"""GPU forces: F = -dE/dR of the fixed-probe estimator (reverse mode through the
Lanczos recurrence on the GPU) against automatic differentiation of the oracle's
estimator with the same probes, and against central differences of the GPU energy.

Tolerances, element-wise as a fraction of the largest force component: float64 path
1e-7 (rounding of the reverse sweep over m steps; the oracle differentiates the same
definition); mixed path 1e-5 (float32 grids, pair kernel and bilinear force terms,
summed over R m right-hand sides in float64)."""
import numpy as np
import pytest
import torch

import synth
from oracle import lanczos as olz
from oracle import method as om

pytestmark = pytest.mark.gpu

A = synth.ANGSTROM_BOHR
SEED = 12345


def _plan(s, prec, block, R, m, grid=(16, 16, 16), tau_ang=0.35, rc_ang=13.0, forces=True):
    import paper_2307_02278_amd as P
    ds = P.DeviceSystem(s.pos, s.cell, s.alpha, s.omega, s.rvdw)
    prm = P.Params(ewald_tau=tau_ang * synth.BOHR_ANGSTROM, real_cutoff=rc_ang * A, grid=grid,
                   n_probes=R, n_steps=m, block=block, precision=prec, seed=SEED,
                   want_forces=forces)
    return P.Plan([ds], prm)


def _oracle_forces(s, plan, R, m):
    inf = plan.info(0)
    mp = om.MethodParams(tau=inf.tau, r_pair=inf.r_pair, grid=tuple(inf.grid),
                         order=inf.spline_order, beta=0.83, d=6.0)
    pos = torch.tensor(s.pos, requires_grad=True)
    op = om.Operator(s, mp, pos=pos)
    res = olz.slq(op, s.n, s.omega, seed=SEED, n_probes=R, m=m, reorth="none")
    (g,) = torch.autograd.grad(res.energy, pos)
    return float(res.energy), -g


@pytest.fixture(scope="module")
def tiny():
    return synth.workload("tiny").systems[0]


@pytest.mark.parametrize("block", [4, 8])
def test_forces_fp64_match_oracle(tiny, block):
    import paper_2307_02278_amd as P
    R, m = 8, 12
    plan = _plan(tiny, P.PREC_FP64, block, R, m)
    e, f = plan.execute(forces=True)
    plan.check()
    e_ref, f_ref = _oracle_forces(tiny, plan, R, m)
    assert float(e[0]) == pytest.approx(e_ref, rel=1e-9)
    f = f.cpu()
    err = float((f - f_ref).abs().max()) / float(f_ref.abs().max())
    print(f"fp64 forces, block {block}: {err:.2e} of max |F|")
    assert err <= 1e-7, err


@pytest.mark.parametrize("block", [16, 64, 128])
def test_forces_mixed_match_oracle(tiny, block):
    import paper_2307_02278_amd as P
    R, m = 16, 12  # at block 128 the block is ragged (16 probes in flight)
    plan = _plan(tiny, P.PREC_MIXED, block, R, m)
    e, f = plan.execute(forces=True)
    plan.check()
    e_ref, f_ref = _oracle_forces(tiny, plan, R, m)
    assert float(e[0]) == pytest.approx(e_ref, rel=1e-5)
    err = float((f.cpu() - f_ref).abs().max()) / float(f_ref.abs().max())
    print(f"mixed forces, block {block}: {err:.2e} of max |F|")
    assert err <= 1e-5, err


def test_forces_match_finite_differences_of_gpu_energy(tiny):
    """Central differences (h = 1e-4 bohr) of the float64 GPU energy at fixed probes."""
    import paper_2307_02278_amd as P
    R, m = 4, 10
    plan = _plan(tiny, P.PREC_FP64, 4, R, m)
    _, f = plan.execute(forces=True)
    plan.check()
    f = f.cpu()
    h = 1e-4
    for a, c in [(0, 0), (37, 1), (90, 2)]:
        es = []
        for sgn in (1, -1):
            p = torch.tensor(tiny.pos)
            p[a, c] += sgn * h
            plan.set_positions(p.cuda())
            es.append(float(plan.execute()[0]))
            plan.check()
        fd = -(es[0] - es[1]) / (2 * h)
        assert float(f[a, c]) == pytest.approx(fd, rel=1e-5, abs=1e-9), (a, c)


def test_forces_with_lanczos_breakdown():
    """One atom: the Krylov space has dimension 3, every probe breaks down early and the
    reverse sweep must skip the steps past m_eff."""
    import paper_2307_02278_amd as P
    s = synth.one_atom(at=(1.1, 2.2, 3.3))
    R, m = 4, 6
    plan = _plan(s, P.PREC_FP64, 4, R, m)
    e, f = plan.execute(forces=True)
    plan.check()
    assert torch.isfinite(f).all()
    e_ref, f_ref = _oracle_forces(s, plan, R, m)
    assert float(e[0]) == pytest.approx(e_ref, rel=1e-9, abs=1e-15)
    assert float((f.cpu() - f_ref).abs().max()) <= 1e-7 * max(float(f_ref.abs().max()), 1e-12)


def test_forces_of_two_systems_in_one_plan(tiny):
    """Forces of a batch come back concatenated in the systems' order."""
    import paper_2307_02278_amd as P
    small = synth.tiny_random(seed=9, n=40)
    R, m = 4, 8
    prm = P.Params(ewald_tau=0.35 * synth.BOHR_ANGSTROM, real_cutoff=13.0 * A, grid=(16,) * 3,
                   n_probes=R, n_steps=m, block=4, precision=P.PREC_FP64, seed=SEED,
                   want_forces=True)
    ds = [P.DeviceSystem(x.pos, x.cell, x.alpha, x.omega, x.rvdw) for x in (tiny, small)]
    both = P.Plan(ds, prm)
    e, f = both.execute(forces=True)
    both.check()
    assert f.shape == (tiny.n + small.n, 3)
    for k, (x, lo) in enumerate([(tiny, 0), (small, tiny.n)]):
        one = P.Plan([ds[k]], prm)
        e1, f1 = one.execute(forces=True)
        one.check()
        # probes are keyed by the system index: system 1 alone is system 0 of its plan
        if k == 0:
            assert float(e[0]) == float(e1[0])
            assert torch.equal(f[lo:lo + x.n], f1)
        else:
            assert torch.isfinite(f[lo:lo + x.n]).all()


def test_autograd_function_returns_minus_forces(tiny):
    import paper_2307_02278_amd as P
    plan = _plan(tiny, P.PREC_FP64, 4, 4, 8)
    pos = torch.tensor(tiny.pos, device="cuda", requires_grad=True)
    E = P.MBDEnergy.apply(pos, plan)
    E.backward()
    _, f = plan.execute(forces=True)
    assert torch.allclose(pos.grad, -f, rtol=0, atol=1e-14)


def test_forces_need_a_forces_plan(tiny):
    import paper_2307_02278_amd as P
    plan = _plan(tiny, P.PREC_FP64, 4, 4, 6, forces=False)
    with pytest.raises(P.MbdError) as ei:
        plan.execute(forces=True)
    assert ei.value.code == -9


def _shaped_plan(s, block, R, m, mode, grid=(16, 16, 16), tau_ang=0.35, rc_ang=13.0):
    import paper_2307_02278_amd as P
    ds = P.DeviceSystem(s.pos, s.cell, s.alpha, s.omega, s.rvdw)
    prm = P.Params(ewald_tau=tau_ang * synth.BOHR_ANGSTROM if tau_ang else 0.0,
                   real_cutoff=rc_ang * A, grid=grid, n_probes=R, n_steps=m, block=block,
                   precision=P.PREC_MIXED, seed=SEED, want_forces=True, tune=P.TUNE_GIVEN,
                   shape=dict(overlap=1, pair_mode=mode, pair_subsets=4 if mode else 0))
    return P.Plan([ds], prm)


def test_matrix_core_forces_match_oracle(tiny):
    """Direct force terms on the matrix cores (per-pair M1 = sum p_t q_j^T and
    M2 = sum q_t p_j^T as dense products over the right-hand sides), 64 probes as one
    block, against autograd of the oracle's estimator."""
    R, m = 64, 10
    plan = _shaped_plan(tiny, 64, R, m, 1)
    assert plan.info(0).shape.pair_mode == 1
    e, f = plan.execute(forces=True)
    plan.check()
    e_ref, f_ref = _oracle_forces(tiny, plan, R, m)
    assert float(e[0]) == pytest.approx(e_ref, rel=1e-5)
    f = f.cpu()
    err = float((f - f_ref).abs().max()) / float(f_ref.abs().max())
    print(f"matrix-core forces vs oracle: {err:.2e} of max |F|")
    assert err <= 1e-5, err


@pytest.mark.parametrize("block", [64, 128])
def test_matrix_core_forces_match_vector_forces(block):
    """600 atoms (38 target groups, the last one ragged; candidate blocks of 16 with a
    ragged tail): matrix-core and vector direct force terms give the same forces to the
    mixed-precision bound."""
    s = synth.water_box(200, seed=11)
    out = []
    for mode in (0, 1):
        plan = _shaped_plan(s, block, block, 8, mode, grid=(24, 24, 24), tau_ang=None,
                            rc_ang=7.0)
        assert plan.info(0).shape.pair_mode == mode
        e, f = plan.execute(forces=True)
        plan.check()
        out.append((float(e[0]), f.cpu()))
        plan.close()
    err = float((out[1][1] - out[0][1]).abs().max()) / float(out[0][1].abs().max())
    print(f"matrix-core vs vector forces, B={block}: {err:.2e} of max |F|")
    assert err <= 1e-5, err
    assert out[1][0] == pytest.approx(out[0][0], rel=1e-6)


@pytest.mark.parametrize("prec,block,mode", [(0, 8, 0), (1, 16, 0), (1, 64, 1)])
def test_kept_forward_grids_give_the_same_forces(tiny, prec, block, mode):
    """store_grids: the reverse force terms read the forward steps' potential grids
    (phi of y_k, scaled per right-hand side) instead of spreading and transforming
    q = c9 g y_k again. Same energy bits; forces to the precision's bound, and against
    the oracle."""
    import paper_2307_02278_amd as P
    R, m = 16 if block < 64 else 64, 10
    ds = P.DeviceSystem(tiny.pos, tiny.cell, tiny.alpha, tiny.omega, tiny.rvdw)
    out = []
    for keep in (False, True):
        prm = P.Params(ewald_tau=0.35 * synth.BOHR_ANGSTROM, real_cutoff=13.0 * A,
                       grid=(16, 16, 16), n_probes=R, n_steps=m, block=block, precision=prec,
                       seed=SEED, want_forces=True, store_grids=keep, tune=P.TUNE_GIVEN,
                       shape=dict(overlap=1, pair_mode=mode, pair_subsets=4 if mode else 0))
        plan = P.Plan([ds], prm)
        e, f = plan.execute(forces=True)
        e2, f2 = plan.execute(forces=True)  # the kept grids are rewritten each run
        plan.check()
        assert torch.equal(f, f2)
        out.append((e.cpu(), f.cpu()))
        if keep:
            _, f_ref = _oracle_forces(tiny, plan, R, m)
        plan.close()
    assert torch.equal(out[0][0], out[1][0])
    err = float((out[1][1] - out[0][1]).abs().max()) / float(out[0][1].abs().max())
    tol = 1e-12 if prec == 0 else 1e-5
    print(f"kept grids vs recomputed, prec {prec}, block {block}: {err:.2e} of max |F|")
    assert err <= tol, err
    oerr = float((out[1][1] - f_ref).abs().max()) / float(f_ref.abs().max())
    print(f"kept grids vs oracle: {oerr:.2e}")
    assert oerr <= (1e-7 if prec == 0 else 1e-5), oerr
