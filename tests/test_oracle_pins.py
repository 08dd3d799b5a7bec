"""Pins for the CPU oracle: closed forms, invariants, published values and
brute force, each independent of the oracle's own formulas."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import dense, exact, lanczos, method, params, probes, replica, spme
from tests.conftest import read_golden

A = synth.ANGSTROM_BOHR
BETA, DAMP = 0.83, 6.0


@pytest.fixture(scope="module")
def tiny():
    return synth.tiny_random(seed=1)


@pytest.fixture(scope="module")
def tiny_C(tiny):
    return exact.coupling_dense(tiny, 0.35 * synth.BOHR_ANGSTROM, BETA, DAMP)


# --- published values -------------------------------------------------------

def test_tau_rule_reproduces_paper_value():
    rc, tau = map(float, read_golden("tau_rule.txt")[0])
    # agrees with the printed six decimals to within one unit of the last digit
    assert abs(params.tau_from_cutoff_angstrom(rc) - tau) < 1e-6


def test_splitmix64_published_outputs():
    want = [int(r[0], 16) for r in read_golden("splitmix64_seed0.txt")]
    got = [int(x) for x in probes.splitmix64(0, np.arange(len(want)))]
    assert got == want


def test_bspline_textbook_values():
    for x, v in read_golden("bspline_m4.txt"):
        assert float(spme.bspline(4, torch.tensor([float(x)], dtype=torch.float64))) == \
            pytest.approx(float(v), abs=1e-15)


def test_grid_rule_matches_workload_grids():
    assert params.smooth_grid(10.0) == 16
    assert params.smooth_grid(31.04) == 48
    assert params.smooth_grid(62.09) == 96


# --- probes (eq. dds) -----------------------------------------------------------

def test_probes_are_normalized_rademacher():
    V = probes.rademacher(12345, 0, 500, range(4))
    D = 1500
    assert torch.allclose(V.abs(), torch.full_like(V, 1 / math.sqrt(D)))
    assert torch.allclose((V.reshape(4, -1) ** 2).sum(1), torch.ones(4, dtype=torch.float64))
    frac_pos = float((V > 0).double().mean())
    assert abs(frac_pos - 0.5) < 0.02
    # distinct systems and probes draw different signs
    W = probes.rademacher(12345, 1, 500, range(4))
    assert not torch.equal(V, W)
    assert not torch.equal(V[0], V[1])


# --- B-splines and exponential interpolation (eqs. scaledfractional, spme) ---

@pytest.mark.parametrize("p", [4, 6, 8])
def test_bspline_partition_of_unity_and_derivative(p):
    w = torch.rand(200, dtype=torch.float64)
    t = torch.arange(p, dtype=torch.float64)
    x = w[:, None] + t[None, :]
    assert torch.allclose(spme.bspline(p, x).sum(1), torch.ones(200, dtype=torch.float64),
                          atol=1e-14)
    assert torch.allclose(spme.bspline_deriv(p, x).sum(1), torch.zeros(200, dtype=torch.float64),
                          atol=1e-14)
    h = 1e-6
    fd = (spme.bspline(p, x + h) - spme.bspline(p, x - h)) / (2 * h)
    assert torch.allclose(fd, spme.bspline_deriv(p, x), atol=1e-8)
    # symmetric about p/2
    xs = torch.linspace(0.01, p - 0.01, 101, dtype=torch.float64)
    assert torch.allclose(spme.bspline(p, xs), spme.bspline(p, p - xs), atol=1e-14)


@pytest.mark.parametrize("p", [4, 6, 8])
def test_euler_spline_interpolates_exponentials(p):
    """b(m) sum_k M_p(u - k) e^{2 pi i m k / K} approximates e^{2 pi i m u / K}."""
    K = 32
    u = torch.rand(50, dtype=torch.float64) * K
    k = torch.arange(-p - 2, K + p + 2, dtype=torch.float64)
    errs = []
    for m in (1, 2, 4):
        # b(m) with its phase: e^{2 pi i (p-1) m / K} / sum_{k=0}^{p-2} M_p(k+1) e^{2 pi i m k / K}
        kk = torch.arange(p - 1, dtype=torch.float64)
        den = (spme.bspline(p, kk + 1) * torch.exp(2j * math.pi * m * kk / K)).sum()
        b = torch.exp(torch.tensor(2j * math.pi * (p - 1) * m / K, dtype=torch.complex128)) / den
        assert abs(abs(b) ** 2 - float(spme.bmod2(p, K)[m])) < 1e-12
        W = spme.bspline(p, u[:, None] - k[None, :])
        approx = b * (W * torch.exp(2j * math.pi * m * k / K)[None, :]).sum(1)
        exact_v = torch.exp(2j * math.pi * m * u / K)
        errs.append(float((approx - exact_v).abs().max()))
    assert errs[0] < 10 ** (-p / 2.0)
    assert errs[0] < errs[1] < errs[2]


# --- the exact periodic tensor (eqs. replica, ewalddip, fld_ewald, fld_ewald1, fld_ewald2) --

def test_ewald_tau_independence(tiny):
    Ts = [exact.tpbc_dense(tiny.pos, tiny.cell, t * synth.BOHR_ANGSTROM, tiny.rvdw, BETA, DAMP)
          for t in (0.25, 0.35, 0.50)]
    for T in Ts[1:]:
        assert float((T - Ts[0]).norm() / Ts[0].norm()) < 1e-12


def test_printed_self_coefficient_breaks_tau_independence(tiny):
    """The printed self coefficient 2 tau^3/(3 sqrt pi) would leave a tau-dependent diagonal."""
    t1, t2 = 0.25 * synth.BOHR_ANGSTROM, 0.5 * synth.BOHR_ANGSTROM
    T1 = exact.tpbc_dense(tiny.pos, tiny.cell, t1, tiny.rvdw, BETA, DAMP)
    T2 = exact.tpbc_dense(tiny.pos, tiny.cell, t2, tiny.rvdw, BETA, DAMP)
    shift = lambda t: (4 - 2) * t ** 3 / (3 * math.sqrt(math.pi))  # printed minus used, per unit
    D1 = T1 + shift(t1) * torch.eye(T1.shape[0], dtype=torch.float64)
    D2 = T2 + shift(t2) * torch.eye(T2.shape[0], dtype=torch.float64)
    assert float((D1 - D2).norm() / T1.norm()) > 1e-3


@pytest.mark.parametrize("at", [(0.0, 0.0, 0.0), (1.37, 4.2, 8.9)])
def test_one_atom_closed_form(at):
    alpha, omega, L, E_ref = map(float, read_golden("one_atom.txt")[0])
    s = synth.one_atom(alpha=alpha, omega=omega, L_ang=L, at=at)
    V = (L * A) ** 3
    T = exact.tpbc_dense(s.pos, s.cell, 0.35 * synth.BOHR_ANGSTROM, s.rvdw, BETA, DAMP)
    assert torch.allclose(T, -4 * math.pi / (3 * V) * torch.eye(3, dtype=torch.float64),
                          rtol=1e-12, atol=1e-18)
    C = exact.coupling_dense(s, 0.35 * synth.BOHR_ANGSTROM, BETA, DAMP)
    E = float(dense.energy_from_C(C, s.omega))
    assert E == pytest.approx(E_ref, rel=2e-4)
    assert E == pytest.approx(1.5 * omega * (math.sqrt(1 - 4 * math.pi * alpha / (3 * V)) - 1),
                              rel=1e-12)


def test_simple_cubic_uniform_mode():
    a = 3.0
    s = synth.simple_cubic(3, a)
    tau = 0.4 * synth.BOHR_ANGSTROM
    C = exact.coupling_dense(s, tau, BETA, DAMP)
    u = torch.zeros(s.n, 3, dtype=torch.float64)
    u[:, 0] = 1.0
    lam = s.omega[0] ** 2 * (1 - 4 * math.pi * s.alpha[0] / (3 * (a * A) ** 3))
    Cu = (C @ u.reshape(-1)).reshape(s.n, 3)
    assert torch.allclose(Cu, lam * u, atol=1e-13)


def test_block_trace_is_minus_four_pi_over_volume(tiny):
    T = exact.tpbc_dense(tiny.pos, tiny.cell, 0.35 * synth.BOHR_ANGSTROM, tiny.rvdw, BETA, DAMP)
    N = tiny.n
    V = abs(np.linalg.det(tiny.cell))
    tr = T.reshape(N, 3, N, 3).diagonal(dim1=1, dim2=3).sum(-1)
    assert float((tr + 4 * math.pi / V).abs().max()) < 1e-12 * 4 * math.pi / V * 1e3


def test_coupling_symmetric_positive_definite(tiny_C):
    assert float((tiny_C - tiny_C.T).abs().max()) < 1e-15
    assert float(torch.linalg.eigvalsh(tiny_C).min()) > 0.0


def test_translation_and_permutation_invariance(tiny, tiny_C):
    tau = 0.35 * synth.BOHR_ANGSTROM
    shifted = synth.System("t", tiny.pos + np.array([1.3, -2.1, 0.7]), tiny.cell,
                           tiny.alpha, tiny.omega, tiny.rvdw)
    C2 = exact.coupling_dense(shifted, tau, BETA, DAMP)
    assert float((C2 - tiny_C).abs().max()) < 1e-13
    perm = np.random.default_rng(0).permutation(tiny.n)
    P = synth.System("p", tiny.pos[perm], tiny.cell, tiny.alpha[perm], tiny.omega[perm],
                     tiny.rvdw[perm])
    C3 = exact.coupling_dense(P, tau, BETA, DAMP)
    idx = torch.from_numpy(np.repeat(perm * 3, 3) + np.tile(np.arange(3), tiny.n))
    assert float((C3 - tiny_C[idx][:, idx]).abs().max()) < 1e-13


def test_matrix_free_exact_matches_dense(tiny, tiny_C):
    y = torch.randn(tiny.n, 3, 2, dtype=torch.float64, generator=torch.Generator().manual_seed(3))
    got = exact.matvec_exact(tiny, 0.35 * synth.BOHR_ANGSTROM, BETA, DAMP, y)
    want = (tiny_C @ y.reshape(-1, 2)).reshape(tiny.n, 3, 2)
    assert float((got - want).norm() / want.norm()) < 1e-13
    sub = torch.tensor([0, 7, 50, 95])
    part = exact.matvec_exact(tiny, 0.35 * synth.BOHR_ANGSTROM, BETA, DAMP, y, targets=sub)
    assert torch.allclose(part, want[sub], rtol=0, atol=1e-13 * float(want.abs().max()))


def test_dimer_free_space_and_london_limit():
    for r_ang in (3.0, 6.0):
        s = synth.dimer(r_ang)
        C = exact.coupling_free(s, BETA, DAMP)
        r = r_ang * A
        S = BETA * 2 * s.rvdw[0]
        f = 1 / (1 + math.exp(-DAMP * (r / S - 1)))
        w2, al = s.omega[0] ** 2, s.alpha[0]
        tv = [-2 / r ** 3, 1 / r ** 3, 1 / r ** 3]
        want = sorted(w2 * (1 + sg * al * f * t) for t in tv for sg in (1, -1))
        got = sorted(float(x) for x in torch.linalg.eigvalsh(C))
        assert np.allclose(got, want, rtol=1e-13)
        # periodic box of 200 A differs from free space only by far images
        Cp = exact.coupling_dense(s, 0.35 * synth.BOHR_ANGSTROM, BETA, DAMP)
        assert float((Cp - C).abs().max()) < 1e-6 * w2
    # London: E -> -(3/4) omega alpha^2 / r^6 at large r (f -> 1)
    r_ang = 40.0
    s = synth.dimer(r_ang, L_ang=400.0)
    E = float(dense.energy_from_C(exact.coupling_free(s, BETA, DAMP), s.omega))
    r = r_ang * A
    assert E == pytest.approx(-0.75 * s.omega[0] * s.alpha[0] ** 2 / r ** 6, rel=1e-4)


def test_replica_sum_tends_to_ewald_plus_surface_term(tiny):
    """Spherical replica sums converge (slowly) to the vacuum limit T^pbc + 4 pi/(3V)."""
    tau = 0.35 * synth.BOHR_ANGSTROM
    N = tiny.n
    V = abs(np.linalg.det(tiny.cell))
    L = tiny.cell[0, 0]
    g = torch.from_numpy(tiny.omega * np.sqrt(tiny.alpha))
    dv = torch.randn(N, 3, 1, dtype=torch.float64, generator=torch.Generator().manual_seed(5))
    E_ew = exact.matvec_exact(tiny, tau, BETA, DAMP, dv / g[:, None, None],
                              components=2 | 4 | 8) / g[:, None, None]
    surf = 4 * math.pi / (3 * V) * dv.sum(0, keepdim=True)
    errs = []
    for k in (1, 2, 4):
        Er = replica.replica_field(tiny, BETA, DAMP, k * L, dv)
        errs.append(float((Er - surf - E_ew).norm() / E_ew.norm()))
    no_surface = float((Er - E_ew).norm() / E_ew.norm())
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-2
    assert no_surface > 0.1


# --- the SPME method operator ----------------------------------------------------

def test_spme_converges_to_exact_ewald(tiny, tiny_C):
    tau = 0.35 * synth.BOHR_ANGSTROM
    y = torch.randn(tiny.n, 3, 2, dtype=torch.float64, generator=torch.Generator().manual_seed(7))
    want = (tiny_C @ y.reshape(-1, 2)).reshape(tiny.n, 3, 2)
    errs = []
    for K in (8, 12, 16, 24, 32):
        op = method.Operator(tiny, method.MethodParams(tau=tau, r_pair=13 * A, grid=(K, K, K)))
        errs.append(float((op(y) - want).norm() / want.norm()))
    assert all(e1 > e2 for e1, e2 in zip(errs, errs[1:]))
    assert errs[-1] < 1e-7
    # higher spline order converges faster at a fixed grid
    perr = []
    for p in (4, 6, 8):
        op = method.Operator(tiny, method.MethodParams(tau=tau, r_pair=13 * A, grid=(16,) * 3,
                                                       order=p))
        perr.append(float((op(y) - want).norm() / want.norm()))
    assert perr[0] > perr[1] > perr[2]


def test_spme_reciprocal_matches_structure_factor_sum(tiny):
    tau = 0.35 * synth.BOHR_ANGSTROM
    d = torch.randn(tiny.n, 3, 1, dtype=torch.float64, generator=torch.Generator().manual_seed(9))
    pos = torch.as_tensor(tiny.pos)
    got = spme.recip_field(pos, tiny.cell, [32] * 3, 8, tau, d)
    g = torch.from_numpy(tiny.omega * np.sqrt(tiny.alpha))
    want = exact.matvec_exact(tiny, tau, BETA, DAMP, d / g[:, None, None], components=4) / \
        g[:, None, None]
    assert float((got - want).norm() / want.norm()) < 1e-7


def test_spme_operator_symmetric_and_translation_stable(tiny):
    tau = 0.35 * synth.BOHR_ANGSTROM
    mp = method.MethodParams(tau=tau, r_pair=13 * A, grid=(16,) * 3)
    op = method.Operator(tiny, mp)
    gen = torch.Generator().manual_seed(11)
    u = torch.randn(tiny.n, 3, dtype=torch.float64, generator=gen)
    v = torch.randn(tiny.n, 3, dtype=torch.float64, generator=gen)
    assert abs(float((u * op(v)).sum() - (v * op(u)).sum())) < 1e-14 * float(op(u).norm())
    moved = synth.System("m", tiny.pos + np.array([0.31, 0.77, -1.9]), tiny.cell, tiny.alpha,
                         tiny.omega, tiny.rvdw)
    op2 = method.Operator(moved, mp)
    assert float((op2(v) - op(v)).norm() / op(v).norm()) < 1e-5


def test_method_direct_part_matches_exact_at_converged_cutoff(tiny):
    tau = 0.35 * synth.BOHR_ANGSTROM
    S = BETA * 2 * tiny.rvdw.max()
    mp = method.MethodParams(tau=tau, r_pair=max(6 / tau, 7.2 * S), grid=(8,) * 3)
    op = method.Operator(tiny, mp)
    y = torch.randn(tiny.n, 3, dtype=torch.float64, generator=torch.Generator().manual_seed(13))
    want = exact.matvec_exact(tiny, tau, BETA, DAMP, y, components=2)
    assert float((op(y, method.DIR) - want).norm() / want.norm()) < 1e-13


# --- Lanczos quadrature (eqs. sl1-sl4, tridiag1, recurs) ---------------------------

def test_full_krylov_quadrature_is_exact(tiny, tiny_C):
    N = tiny.n
    v = probes.rademacher(12345, 0, N, [0])[0]
    mv = lambda x: (tiny_C @ x.reshape(-1)).reshape(x.shape)
    res = lanczos.lanczos(mv, v, 3 * N)
    q, theta, wts = lanczos.quadrature(res.a, res.b)
    assert float(q) == pytest.approx(float(dense.sqrt_trace_probe(tiny_C, v)), rel=1e-12)
    assert float(wts.sum()) == pytest.approx(1.0, abs=1e-13)
    lam = torch.linalg.eigvalsh(tiny_C)
    assert float(theta.min()) >= float(lam.min()) - 1e-12
    assert float(theta.max()) <= float(lam.max()) + 1e-12


def test_lanczos_tridiagonal_is_projection(tiny, tiny_C):
    v = probes.rademacher(12345, 0, tiny.n, [1])[0]
    mv = lambda x: (tiny_C @ x.reshape(-1)).reshape(x.shape)
    res = lanczos.lanczos(mv, v, 20)
    Y = res.Y
    assert torch.allclose(Y @ Y.T, torch.eye(20, dtype=torch.float64), atol=1e-13)
    assert torch.allclose(Y @ tiny_C @ Y.T, lanczos.tridiagonal(res.a, res.b), atol=1e-13)


def test_fifteen_steps_suffice(tiny, tiny_C):
    """Krylov dimension 15 already gives the quadrature to ~1e-11 (Numerical results)."""
    mv = lambda x: (tiny_C @ x.reshape(-1)).reshape(x.shape)
    for l in range(3):
        v = probes.rademacher(12345, 0, tiny.n, [l])[0]
        q15 = lanczos.quadrature(*[getattr(lanczos.lanczos(mv, v, 15), k) for k in ("a", "b")])[0]
        q40 = lanczos.quadrature(*[getattr(lanczos.lanczos(mv, v, 40), k) for k in ("a", "b")])[0]
        assert abs(float(q15 - q40)) < 1e-10 * abs(float(q40))


def test_hutchinson_estimate_is_unbiased(tiny, tiny_C):
    N = tiny.n
    mv = lambda x: (tiny_C @ x.reshape(-1, x.shape[-1] if x.dim() == 3 else 1)).reshape(x.shape)
    op = lambda y: (tiny_C @ y.reshape(-1)).reshape(y.shape)
    res = lanczos.slq(op, N, tiny.omega, seed=777, n_probes=64, m=20)
    est = res.q * 3 * N
    exact_tr = float(torch.sqrt(torch.linalg.eigvalsh(tiny_C)).sum())
    sd = float(est.std()) / math.sqrt(len(est))
    assert abs(float(est.mean()) - exact_tr) < 4 * sd
    E_exact = float(dense.energy_from_C(tiny_C, tiny.omega))
    assert abs(float(res.energy) - E_exact) < 2 * sd


def test_decoupled_limit_gives_zero_energy(tiny):
    """alpha -> 0 leaves C = Omega; with three distinct omegas the Krylov space has
    dimension 3, Lanczos breaks down there, the quadrature is exact and E = 0."""
    om = np.array([0.3, 0.45, 0.7])[np.arange(tiny.n) % 3]
    s = synth.System("z", tiny.pos, tiny.cell, np.full(tiny.n, 1e-300), om, tiny.rvdw)
    op = method.Operator(s, method.MethodParams(tau=0.35 * synth.BOHR_ANGSTROM, r_pair=13 * A,
                                                grid=(8,) * 3))
    res = lanczos.slq(op, s.n, s.omega, seed=1, n_probes=4, m=6)
    assert all(len(a) == 3 for a in res.a)
    assert abs(float(res.energy)) < 1e-13


# --- gradients (forces are future work in the paper; defined as -dE/dR) -------------

def test_exact_energy_gradient_matches_finite_differences():
    s = synth.tiny_random(seed=1)
    s = synth.System("s", s.pos[:24], s.cell, s.alpha[:24], s.omega[:24], s.rvdw[:24])
    tau = 0.35 * synth.BOHR_ANGSTROM
    pos = torch.tensor(s.pos, requires_grad=True)
    E = dense.energy_from_C(exact.coupling_dense(s, tau, BETA, DAMP, pos=pos), s.omega)
    (g,) = torch.autograd.grad(E, pos)
    h = 1e-4
    for a, c in [(0, 0), (5, 1), (17, 2)]:
        pp, pm = s.pos.copy(), s.pos.copy()
        pp[a, c] += h
        pm[a, c] -= h
        Ep = dense.energy_from_C(exact.coupling_dense(s, tau, BETA, DAMP, pos=pp), s.omega)
        Em = dense.energy_from_C(exact.coupling_dense(s, tau, BETA, DAMP, pos=pm), s.omega)
        assert float(g[a, c]) == pytest.approx(float(Ep - Em) / (2 * h), rel=1e-6, abs=2e-10)
    assert float(g.sum(0).abs().max()) < 1e-12 * float(g.abs().max()) * 1e3


def test_fixed_seed_slq_gradient_matches_finite_differences(tiny):
    tau = 0.35 * synth.BOHR_ANGSTROM
    mp = method.MethodParams(tau=tau, r_pair=13 * A, grid=(12,) * 3)

    def energy(p):
        op = method.Operator(tiny, mp, pos=p)
        return lanczos.slq(op, tiny.n, tiny.omega, seed=3, n_probes=2, m=8).energy

    pos = torch.tensor(tiny.pos, requires_grad=True)
    (g,) = torch.autograd.grad(energy(pos), pos)
    h = 1e-4
    for a, c in [(1, 0), (40, 2)]:
        pp, pm = torch.tensor(tiny.pos), torch.tensor(tiny.pos)
        pp[a, c] += h
        pm[a, c] -= h
        fd = (float(energy(pp)) - float(energy(pm))) / (2 * h)
        assert float(g[a, c]) == pytest.approx(fd, rel=1e-5, abs=1e-10)
