"""GPU parity: the HIP path through the C ABI against the CPU oracle on the same
seeded inputs, element by element. A matvec error is, for each right-hand side,
max |got - want| / max |want|, and the largest over the right-hand sides is bounded.
Tolerances: float64 path 1e-11 (rounding of differently ordered sums over up to ~1e4
terms); mixed path (float32 SPME and pair kernel, float64 Omega v, self term and
Lanczos) 1e-6 on C v, the field parts alone at their float32 level (MIXED_TOL), and
1e-5 relative on E_MBD at fixed probes."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import lanczos as olz
from oracle import method as om

pytestmark = pytest.mark.gpu

A = synth.ANGSTROM_BOHR


def _plan(s, prec, block, R=4, m=10, grid=None, tau_ang=None, rc_ang=9.0, reorth=0, seed=12345,
          damp_tol=0.0):
    import paper_2307_02278_amd as P
    ds = P.DeviceSystem(s.pos, s.cell, s.alpha, s.omega, s.rvdw)
    prm = P.Params(ewald_tau=(tau_ang * synth.BOHR_ANGSTROM if tau_ang else 0.0),
                   real_cutoff=rc_ang * A, grid=grid or (0, 0, 0), n_probes=R, n_steps=m,
                   block=block, precision=prec, reorth=reorth, seed=seed, damp_tol=damp_tol)
    return P.Plan([ds], prm), ds


def _oracle_op(s, plan):
    inf = plan.info(0)
    mp = om.MethodParams(tau=inf.tau, r_pair=inf.r_pair, grid=tuple(inf.grid),
                         order=inf.spline_order, beta=0.83, d=6.0)
    return om.Operator(s, mp)


def _err(got, want, label=""):
    """Element-wise error of a block of vectors [nrhs][N][3]: the largest, over the
    right-hand sides, of max |got - want| / max |want| within that right-hand side."""
    num = (got - want).abs().reshape(got.shape[0], -1).amax(1)
    den = want.abs().reshape(want.shape[0], -1).amax(1)
    e = float((num / den).max())
    print(f"element-wise error {label}: {e:.2e}")
    return e


# float32 grids and pair kernel: the whole C v to the 1e-6 bound; single parts of the
# field (no Omega v in them) to their own float32 rounding level
MIXED_TOL = {1: 1e-13, 2: 1e-5, 4: 1e-5, 8: 1e-13, 15: 1e-6}


@pytest.fixture(scope="module")
def tiny():
    return synth.workload("tiny").systems[0]


@pytest.fixture(scope="module")
def rhs4(tiny):
    g = torch.Generator().manual_seed(21)
    return torch.randn(4, tiny.n, 3, dtype=torch.float64, generator=g)


COMPONENTS = [(1, "diag"), (2, "dir"), (4, "rec"), (8, "self"), (15, "all")]


@pytest.mark.parametrize("comp,name", COMPONENTS)
def test_matvec_fp64_components(tiny, rhs4, comp, name):
    import paper_2307_02278_amd as P
    plan, _ = _plan(tiny, P.PREC_FP64, 4, grid=(16, 16, 16), tau_ang=0.35, rc_ang=13.0)
    op = _oracle_op(tiny, plan)
    got = plan.matvec(rhs4.cuda(), components=comp).cpu()
    want = op(rhs4.permute(1, 2, 0), comp).permute(2, 0, 1)
    assert _err(got, want, name) < 1e-11, name


@pytest.mark.parametrize("comp,name", COMPONENTS)
def test_matvec_mixed_components(tiny, rhs4, comp, name):
    import paper_2307_02278_amd as P
    plan, _ = _plan(tiny, P.PREC_MIXED, 4, grid=(16, 16, 16), tau_ang=0.35, rc_ang=13.0)
    op = _oracle_op(tiny, plan)
    got = plan.matvec(rhs4.cuda(), components=comp).cpu()
    want = op(rhs4.permute(1, 2, 0), comp).permute(2, 0, 1)
    assert _err(got, want, name) < MIXED_TOL[comp], name


@pytest.mark.parametrize("block", [1, 2, 16, 32, 64])
def test_matvec_block_layouts_agree(tiny, block):
    """Every RHS block width (direct and tiled pair kernels, grid chunks) gives the same C v."""
    import paper_2307_02278_amd as P
    plan, _ = _plan(tiny, P.PREC_FP64, block, grid=(16, 16, 16), tau_ang=0.35, rc_ang=13.0)
    op = _oracle_op(tiny, plan)
    n = min(block, 3)
    g = torch.Generator().manual_seed(block)
    v = torch.randn(n, tiny.n, 3, dtype=torch.float64, generator=g)
    got = plan.matvec(v.cuda()).cpu()
    want = op(v.permute(1, 2, 0)).permute(2, 0, 1)
    assert _err(got, want, f"block {block}") < 1e-11


@pytest.mark.parametrize("block", [16, 32, 64, 128, 256])
@pytest.mark.parametrize("comp", [2, 15])
def test_matvec_mixed_wide_blocks(tiny, block, comp):
    """Float32 paths used for many right-hand sides (tensor-list pair kernel with 1, 2 or 4
    target subsets per wavefront and 1, 2 or 4 wavefronts per group, register FFT, 64-wide
    grid chunks) against the oracle; r_pair > L/2 exercises several images."""
    import paper_2307_02278_amd as P
    plan, _ = _plan(tiny, P.PREC_MIXED, block, grid=(16, 16, 16), tau_ang=0.35, rc_ang=13.0)
    op = _oracle_op(tiny, plan)
    g = torch.Generator().manual_seed(100 + block)
    v = torch.randn(block, tiny.n, 3, dtype=torch.float64, generator=g)
    got = plan.matvec(v.cuda(), components=comp).cpu()
    want = op(v.permute(1, 2, 0), comp).permute(2, 0, 1)
    assert _err(got, want, f"block {block} comp {comp}") < MIXED_TOL[comp]


@pytest.fixture(scope="module")
def water3k():
    return synth.workload("medium").systems[0]


@pytest.mark.parametrize("prec,block,tol", [(0, 2, 1e-11), (1, 64, 1e-6)])
def test_matvec_water_3000(water3k, prec, block, tol):
    """Medium water box (K=48, r_c=7 A): several cells per axis, many tiles and groups."""
    s = water3k
    plan, _ = _plan(s, prec, block, grid=(48, 48, 48), rc_ang=7.0)
    op = _oracle_op(s, plan)
    n = min(block, 8)
    g = torch.Generator().manual_seed(7)
    v = torch.randn(n, s.n, 3, dtype=torch.float64, generator=g)
    got = plan.matvec(v.cuda()).cpu()
    want = op(v.permute(1, 2, 0)).permute(2, 0, 1)
    assert _err(got, want, f"water3000 prec {prec}") < tol


def test_matvec_noncubic_grid_radix_3_5():
    """Orthorhombic box, K = (20, 24, 30): radices 4, 2, 3 and 5, unequal axes."""
    import paper_2307_02278_amd as P
    base = synth.tiny_random(seed=7, n=60)
    cell = np.diag([10.0, 11.5, 13.0]) * A
    pos = base.pos * np.array([1.0, 1.15, 1.3])
    s = synth.System("ortho", pos, cell, base.alpha[:60], base.omega[:60], base.rvdw[:60])
    plan, _ = _plan(s, P.PREC_FP64, 2, grid=(20, 24, 30), tau_ang=0.35, rc_ang=13.0)
    op = _oracle_op(s, plan)
    v = torch.randn(2, s.n, 3, dtype=torch.float64, generator=torch.Generator().manual_seed(3))
    assert _err(plan.matvec(v.cuda()).cpu(), op(v.permute(1, 2, 0)).permute(2, 0, 1),
                "ortho fp64") < 1e-11


@pytest.mark.parametrize("grid", [(18, 24, 30), (30, 20, 24), (50, 24, 30), (90, 20, 24)])
@pytest.mark.parametrize("comp", [4, 15])
def test_matvec_mixed_noncubic_odd_half_lengths(grid, comp):
    """Float32 grid path with 16 right-hand sides on unequal axes whose x length K1 = 18 or
    30 packs into an odd number (9, 15) of complex points in the real-column x passes;
    the reciprocal part alone (comp 4) isolates the transforms."""
    import paper_2307_02278_amd as P
    base = synth.tiny_random(seed=7, n=60)
    cell = np.diag([10.0, 11.5, 13.0]) * A
    pos = base.pos * np.array([1.0, 1.15, 1.3])
    s = synth.System("ortho", pos, cell, base.alpha[:60], base.omega[:60], base.rvdw[:60])
    plan, _ = _plan(s, P.PREC_MIXED, 16, grid=grid, tau_ang=0.35, rc_ang=13.0)
    op = _oracle_op(s, plan)
    v = torch.randn(16, s.n, 3, dtype=torch.float64, generator=torch.Generator().manual_seed(5))
    got = plan.matvec(v.cuda(), components=comp).cpu()
    want = op(v.permute(1, 2, 0), comp).permute(2, 0, 1)
    assert _err(got, want, f"grid {grid} comp {comp}") < MIXED_TOL[comp]


@pytest.mark.parametrize("k3", [12, 20, 36, 60, 72, 80, 96, 100, 108, 120, 128, 90])
def test_matvec_z_convolution_lengths(k3):
    """The z pass with the convolution (register transform over lane pairs, the lanes
    exchanging values by quad permutations) at lengths from 12 to 128 with radices 2, 3
    and 5: reciprocal part alone, float32 grid, 16 right-hand sides, against the oracle's
    transform."""
    import paper_2307_02278_amd as P
    base = synth.tiny_random(seed=7, n=60)
    cell = np.diag([10.0, 11.5, 13.0]) * A
    pos = base.pos * np.array([1.0, 1.15, 1.3])
    s = synth.System("ortho", pos, cell, base.alpha[:60], base.omega[:60], base.rvdw[:60])
    plan, _ = _plan(s, P.PREC_MIXED, 16, grid=(16, 18, k3), tau_ang=0.35, rc_ang=13.0)
    op = _oracle_op(s, plan)
    v = torch.randn(16, s.n, 3, dtype=torch.float64, generator=torch.Generator().manual_seed(9))
    got = plan.matvec(v.cuda(), components=4).cpu()
    want = op(v.permute(1, 2, 0), 4).permute(2, 0, 1)
    assert _err(got, want, f"K3 {k3}") < MIXED_TOL[4]


def _compare_lanczos(s, prec, block, R, m, tol_q, tol_e, **kw):
    import paper_2307_02278_amd as P
    plan, _ = _plan(s, prec, block, R=R, m=m, **kw)
    e_gpu = float(plan.execute().cpu()[0])
    plan.check()
    a, b, me = plan.tridiagonal()
    q = plan.quadrature()
    op = _oracle_op(s, plan)
    ref = olz.slq(op, s.n, s.omega, seed=12345, n_probes=R, m=m, reorth="full")
    for l in range(R):
        k = min(8, len(ref.a[l]))
        assert torch.allclose(a[l, :k], ref.a[l][:k], rtol=tol_q, atol=0), l
        if k > 1:
            assert torch.allclose(b[l, :k - 1], ref.b[l][:k - 1], rtol=tol_q, atol=0), l
    assert torch.allclose(q, ref.q, rtol=tol_q, atol=0)
    assert e_gpu == pytest.approx(float(ref.energy), rel=tol_e)
    return e_gpu, float(ref.energy)


@pytest.mark.parametrize("block", [1, 8])
def test_energy_fp64_matches_oracle(tiny, block):
    import paper_2307_02278_amd as P
    _compare_lanczos(tiny, P.PREC_FP64, block, R=8, m=30, tol_q=1e-10, tol_e=1e-9,
                     grid=(16, 16, 16), tau_ang=0.35, rc_ang=13.0)


def test_energy_mixed_matches_oracle(tiny):
    import paper_2307_02278_amd as P
    _compare_lanczos(tiny, P.PREC_MIXED, 8, R=8, m=30, tol_q=2e-6, tol_e=1e-5,
                     grid=(16, 16, 16), tau_ang=0.35, rc_ang=13.0)


def test_ragged_probe_blocks(tiny):
    """R = 5 probes in blocks of 4: the last block is partly empty."""
    import paper_2307_02278_amd as P
    _compare_lanczos(tiny, P.PREC_FP64, 4, R=5, m=12, tol_q=1e-10, tol_e=1e-9,
                     grid=(16, 16, 16), tau_ang=0.35, rc_ang=13.0)


def test_one_atom_breaks_down_and_matches_oracle():
    """N = 1: the Krylov space has dimension <= 3, Lanczos stops early (m_eff <= 3)."""
    import paper_2307_02278_amd as P
    s = synth.one_atom(at=(1.1, 2.2, 3.3))
    plan, _ = _plan(s, P.PREC_FP64, 2, R=2, m=6, grid=(16, 16, 16), tau_ang=0.35, rc_ang=13.0)
    e = float(plan.execute().cpu()[0])
    plan.check()
    _, _, me = plan.tridiagonal()
    assert int(me.max()) <= 3
    op = _oracle_op(s, plan)
    ref = olz.slq(op, 1, s.omega, seed=12345, n_probes=2, m=6)
    assert e == pytest.approx(float(ref.energy), rel=1e-9, abs=1e-15)
    V = (10.0 * A) ** 3
    closed = 1.5 * 0.5 * (math.sqrt(1 - 4 * math.pi * 10.0 / (3 * V)) - 1)
    assert e == pytest.approx(closed, rel=1e-3)


def test_reorthogonalization_modes_agree(tiny):
    import paper_2307_02278_amd as P
    es = []
    for ro in (0, 1, 2):
        plan, _ = _plan(tiny, P.PREC_FP64, 4, R=4, m=20, grid=(16, 16, 16), tau_ang=0.35,
                        rc_ang=13.0, reorth=ro)
        es.append(float(plan.execute().cpu()[0]))
        plan.check()
    assert es[1] == pytest.approx(es[0], rel=1e-10)
    assert es[2] == pytest.approx(es[0], rel=1e-10)


def test_set_positions_rebuilds_pair_list():
    """Moving the atoms re-runs the device setup, including the direct-space tensor list."""
    import paper_2307_02278_amd as P
    s0 = synth.workload("medium").systems[0]
    plan, _ = _plan(s0, P.PREC_MIXED, 16, grid=(48, 48, 48), rc_ang=7.0)
    rng = np.random.default_rng(5)
    pos1 = s0.pos + rng.normal(scale=0.1 * A, size=s0.pos.shape)
    plan.set_positions(torch.as_tensor(pos1).cuda())
    s1 = synth.System("moved", pos1, s0.cell, s0.alpha, s0.omega, s0.rvdw)
    op = _oracle_op(s1, plan)
    v = torch.randn(3, s1.n, 3, dtype=torch.float64, generator=torch.Generator().manual_seed(9))
    got = plan.matvec(v.cuda()).cpu()
    plan.check()
    assert _err(got, op(v.permute(1, 2, 0)).permute(2, 0, 1), "moved") < MIXED_TOL[15]


def test_pair_list_overflow_is_reported():
    """Positions far denser than at plan creation overflow the tensor list's capacity: the
    kernels stay within their buffers and check() reports the condition."""
    import paper_2307_02278_amd as P
    rng = np.random.default_rng(11)
    n, L = 600, 60.0
    pos0 = rng.uniform(0, L, size=(n, 3)) * A
    cell = np.eye(3) * L * A
    ones = np.ones(n)
    s0 = synth.System("dilute", pos0, cell, 6.0 * ones, 0.5 * ones, 3.5 * ones)
    plan, _ = _plan(s0, P.PREC_MIXED, 16, grid=(40, 40, 40), rc_ang=6.0)
    plan.check()
    pos1 = rng.uniform(0, 4.0, size=(n, 3)) * A
    plan.set_positions(torch.as_tensor(pos1).cuda())
    plan.matvec(torch.randn(2, n, 3, dtype=torch.float64).cuda())
    with pytest.raises(P.MbdError) as ei:
        plan.check()
    assert ei.value.code == -9


def test_uneven_batch_runs_concurrently_and_matches_oracle():
    """Three systems of different sizes and grids in one plan (they run on separate
    internal streams); each energy matches the oracle with that system's probe stream."""
    import paper_2307_02278_amd as P
    systems = [synth.tiny_random(seed=9, n=40), synth.workload("tiny").systems[0],
               synth.one_atom(at=(2.0, 3.0, 4.0))]
    R, m = 4, 10
    prm = P.Params(ewald_tau=0.35 * synth.BOHR_ANGSTROM, real_cutoff=13.0 * A, grid=(16, 16, 16),
                   n_probes=R, n_steps=m, block=4, precision=P.PREC_FP64, seed=12345)
    ds = [P.DeviceSystem(x.pos, x.cell, x.alpha, x.omega, x.rvdw) for x in systems]
    plan = P.Plan(ds, prm)
    e = plan.execute().cpu()
    plan.check()
    for k, x in enumerate(systems):
        op = _oracle_op(x, plan) if k == 0 else om.Operator(x, om.MethodParams(
            tau=plan.info(k).tau, r_pair=plan.info(k).r_pair, grid=tuple(plan.info(k).grid),
            order=plan.info(k).spline_order, beta=0.83, d=6.0))
        ref = olz.slq(op, x.n, x.omega, seed=12345, n_probes=R, m=m, system=k)
        assert float(e[k]) == pytest.approx(float(ref.energy), rel=1e-9, abs=1e-14), k


@pytest.mark.parametrize("graph", [False, True])
def test_energy_sd_matches_oracle_spread(tiny, graph):
    """sd(E) = 1/2 (3N) s_Q / sqrt(R) from the sample spread s_Q of the per-probe
    quadrature values (eq. hutch averages R independent samples), against the same
    formula applied to the oracle's per-probe values; one probe gives NaN."""
    import paper_2307_02278_amd as P
    R, m = 8, 30
    ds = P.DeviceSystem(tiny.pos, tiny.cell, tiny.alpha, tiny.omega, tiny.rvdw)
    prm = P.Params(ewald_tau=0.35 * synth.BOHR_ANGSTROM, real_cutoff=13.0 * A,
                   grid=(16, 16, 16), n_probes=R, n_steps=m, block=8,
                   precision=P.PREC_FP64, graph=graph)
    plan = P.Plan([ds], prm)
    for _ in range(2 if graph else 1):
        e, sd = plan.execute(energy_sd=True)
    plan.check()
    op = _oracle_op(tiny, plan)
    ref = olz.slq(op, tiny.n, tiny.omega, seed=12345, n_probes=R, m=m, reorth="full")
    want = 0.5 * 3 * tiny.n * float(ref.q.std(unbiased=True)) / math.sqrt(R)
    print(f"sd(E) gpu {float(sd[0]):.6e} oracle {want:.6e}; E {float(e[0]):.8e}")
    assert float(sd[0]) == pytest.approx(want, rel=1e-8)
    one = P.Plan([ds], P.Params(ewald_tau=0.35 * synth.BOHR_ANGSTROM, real_cutoff=13.0 * A,
                                grid=(16, 16, 16), n_probes=1, n_steps=5, block=1,
                                precision=P.PREC_FP64, graph=graph))
    _, sd1 = one.execute(energy_sd=True)
    one.check()
    assert math.isnan(float(sd1[0]))


@pytest.mark.parametrize("grid", [(18, 24, 30), (30, 20, 24), (50, 24, 30), (96, 20, 24)])
@pytest.mark.parametrize("comp", [4, 15])
def test_matvec_line_spread_fused_with_x_transform(grid, comp):
    """The x-line spread fused with the forward x transform (64 right-hand sides per
    chunk, float): unequal axes, odd and even half lengths of the packed x line, against
    the oracle, and bit for bit against the tile spread followed by the x pass."""
    import paper_2307_02278_amd as P
    base = synth.tiny_random(seed=7, n=60)
    cell = np.diag([10.0, 11.5, 13.0]) * A
    pos = base.pos * np.array([1.0, 1.15, 1.3])
    s = synth.System("ortho", pos, cell, base.alpha[:60], base.omega[:60], base.rvdw[:60])
    ds = P.DeviceSystem(s.pos, s.cell, s.alpha, s.omega, s.rvdw)
    out = []
    for mode in (0, 1):
        prm = P.Params(ewald_tau=0.35 * synth.BOHR_ANGSTROM, real_cutoff=13.0 * A, grid=grid,
                       n_probes=64, n_steps=4, block=64, precision=P.PREC_MIXED,
                       tune=P.TUNE_GIVEN, shape=dict(overlap=1, spread_mode=mode))
        plan = P.Plan([ds], prm)
        assert plan.info(0).shape.spread_mode == mode
        v = torch.randn(64, s.n, 3, dtype=torch.float64,
                        generator=torch.Generator().manual_seed(5))
        out.append(plan.matvec(v.cuda(), components=comp).cpu())
        if mode == 1:
            op = _oracle_op(s, plan)
            want = op(v.permute(1, 2, 0), comp).permute(2, 0, 1)
            assert _err(out[1], want, f"line spread grid {grid} comp {comp}") < MIXED_TOL[comp]
        plan.close()
    diff = float((out[1] - out[0]).abs().max() / out[0].abs().max())
    print(f"line spread vs tile spread: {diff:.2e}")
    assert diff <= 1e-6


def test_line_spread_on_a_general_cell():
    """The fused line spread with the chain-rule matrix of a skewed cell."""
    import paper_2307_02278_amd as P
    s = synth.triclinic_random()
    ds = P.DeviceSystem(s.pos, s.cell, s.alpha, s.omega, s.rvdw)
    prm = P.Params(ewald_tau=0.35 * synth.BOHR_ANGSTROM, real_cutoff=13.0 * A,
                   grid=(16, 18, 20), n_probes=64, n_steps=4, block=64, precision=P.PREC_MIXED,
                   tune=P.TUNE_GIVEN, shape=dict(overlap=1, spread_mode=1))
    plan = P.Plan([ds], prm)
    v = torch.randn(64, s.n, 3, dtype=torch.float64, generator=torch.Generator().manual_seed(8))
    got = plan.matvec(v.cuda()).cpu()
    want = _oracle_op(s, plan)(v.permute(1, 2, 0)).permute(2, 0, 1)
    assert _err(got, want, "line spread, skewed cell") < MIXED_TOL[15]


@pytest.fixture(scope="module")
def water600():
    return synth.water_box(200, seed=11)


@pytest.mark.parametrize("block,nk,mcore", [(64, 1, 1), (64, 2, 1), (64, 4, 1), (128, 1, 1),
                                            (128, 2, 1), (128, 4, 1), (256, 1, 1), (256, 2, 1),
                                            (128, 1, 2), (128, 2, 2), (256, 1, 2)])
def test_matvec_matrix_core_pair_kernel(water600, block, nk, mcore):
    """The direct-space sum on the matrix cores (dense per-group product over 16 targets
    x 3 components, 600 atoms: 38 groups, the last one ragged, and candidate lists whose
    3 x count is not a multiple of the 4 rows per instruction), with 128- or 64-column
    wavefronts (pair_mode 1 or 2), against the oracle element by element and against the
    vector list kernel to float32 rounding."""
    import paper_2307_02278_amd as P
    s = water600
    ds = P.DeviceSystem(s.pos, s.cell, s.alpha, s.omega, s.rvdw)
    v = torch.randn(block, s.n, 3, dtype=torch.float64,
                    generator=torch.Generator().manual_seed(17))
    got = {}
    for mode in (0, mcore):
        prm = P.Params(real_cutoff=7.0 * A, grid=(24, 24, 24), n_probes=block, n_steps=4,
                       block=block, precision=P.PREC_MIXED, tune=P.TUNE_GIVEN,
                       shape=dict(overlap=1, pair_mode=mode, pair_subsets=nk if mode else 0))
        plan = P.Plan([ds], prm)
        assert plan.info(0).shape.pair_mode == mode
        got[mode] = {c: plan.matvec(v.cuda(), components=c).cpu() for c in (2, 15)}
        if mode:
            op = _oracle_op(s, plan)
            for c in (2, 15):
                want = op(v.permute(1, 2, 0), c).permute(2, 0, 1)
                assert _err(got[mode][c], want,
                            f"matrix cores mode {mode} B={block} NK={nk} comp {c}") < MIXED_TOL[c]
        plan.check()
        plan.close()
    # two float32 summation orders of the same terms (the same bits when NK = 1)
    d = _err(got[mcore][2], got[0][2], "matrix cores vs vector kernel")
    assert d < MIXED_TOL[2]


def test_matrix_core_pair_kernel_on_a_general_cell():
    """The matrix-core direct sum with a skewed cell (several images per pair)."""
    import paper_2307_02278_amd as P
    s = synth.triclinic_random()
    ds = P.DeviceSystem(s.pos, s.cell, s.alpha, s.omega, s.rvdw)
    prm = P.Params(ewald_tau=0.35 * synth.BOHR_ANGSTROM, real_cutoff=13.0 * A,
                   grid=(16, 18, 20), n_probes=64, n_steps=4, block=64, precision=P.PREC_MIXED,
                   tune=P.TUNE_GIVEN, shape=dict(overlap=1, pair_mode=1, pair_subsets=2))
    plan = P.Plan([ds], prm)
    assert plan.info(0).shape.pair_mode == 1
    v = torch.randn(64, s.n, 3, dtype=torch.float64, generator=torch.Generator().manual_seed(9))
    op = _oracle_op(s, plan)
    for c in (2, 15):
        got = plan.matvec(v.cuda(), components=c).cpu()
        want = op(v.permute(1, 2, 0), c).permute(2, 0, 1)
        assert _err(got, want, f"matrix cores, skewed cell, comp {c}") < MIXED_TOL[c]
    plan.check()


def test_matrix_core_mode_falls_back_where_it_does_not_apply(tiny):
    """pair_mode 1 is kept only for float tensors and blocks of 64, 128, 192 or 256."""
    import paper_2307_02278_amd as P
    ds = P.DeviceSystem(tiny.pos, tiny.cell, tiny.alpha, tiny.omega, tiny.rvdw)
    for prec, block, want in ((P.PREC_MIXED, 32, 0), (P.PREC_FP64, 64, 0),
                              (P.PREC_MIXED, 64, 1)):
        prm = P.Params(real_cutoff=9.0 * A, grid=(0, 0, 0), n_probes=block, n_steps=3,
                       block=block, precision=prec, tune=P.TUNE_GIVEN,
                       shape=dict(overlap=1, pair_mode=1))
        plan = P.Plan([ds], prm)
        assert plan.info(0).shape.pair_mode == want
        plan.close()
