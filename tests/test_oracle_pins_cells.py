"""Pins for the oracle branches that the cubic-cell pins do not reach: the periodic
k-d-tree pair list, and general (triclinic) cells in the converged Ewald sum and in
SPME. Each is checked against something other than the branch itself: brute-force
enumeration of images, properties of the exact periodic tensor that hold in any
cell (tau-independence, the block trace -4 pi / V), the same lattice written with
another basis, a supercell, and the structure-factor sum."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import exact, method, params, spme, tensors

A = synth.ANGSTROM_BOHR
BETA, DAMP = 0.83, 6.0


# --- the periodic k-d-tree pair list (used by every large-box check) -------------

def _keyed(i, j, r, n):
    """Pairs sorted by (i, j); below half the shortest cell edge there is at most one
    image of j within the cutoff of i, so (i, j) identifies the pair."""
    key = i.numpy().astype(np.int64) * n + j.numpy().astype(np.int64)
    order = np.argsort(key, kind="stable")
    return key[order], r.detach().numpy()[order]


def _compare_pair_lists(pos, cell, rc, targets):
    n = pos.shape[0]
    ib, jb, rb = tensors.pair_list_bruteforce(pos, cell, rc, targets=targets)
    ik, jk, rk = tensors.pair_list(pos, cell, rc, targets=targets)
    kb, vb = _keyed(ib, jb, rb, n)
    kk, vk = _keyed(ik, jk, rk, n)
    assert len(np.unique(kb)) == len(kb)        # one image per (i, j) below L/2
    assert np.array_equal(kb, kk)
    assert np.abs(vb - vk).max() <= 1e-14 * float(np.abs(cell).max())
    return len(kb)


@pytest.fixture(scope="module")
def water3000():
    return synth.water_box(1000, seed=2)


def test_kdtree_pair_list_matches_bruteforce_water_box(water3000):
    """The 3000-atom water box at its pair cutoff (7 A erfc cutoff; damping tail to
    1e-4 gives r_pair = 8.02 A), targets queried by ball (the partial-row path)."""
    s = water3000
    pos = torch.as_tensor(s.pos)
    rc = params.damping_range(BETA * 2 * s.rvdw.max(), DAMP, 1e-4)
    assert 7.0 * A < rc < 0.5 * s.cell[0, 0]
    targets = np.arange(0, s.n, 10)
    npairs = _compare_pair_lists(pos, s.cell, rc, targets)
    # about 0.1 atoms / A^3 x 4/3 pi r^3 neighbours per target
    assert 150 * len(targets) < npairs < 350 * len(targets)


def test_kdtree_all_pairs_path_matches_bruteforce(water3000):
    """The all-pairs path (query_pairs, both directions) restricted to a target subset."""
    s = water3000
    pos = torch.as_tensor(s.pos)
    rc = 7.0 * A
    i, j, r = tensors.pair_list(pos, s.cell, rc)
    targets = np.arange(3, s.n, 37)
    keep = torch.from_numpy(np.isin(i.numpy(), targets))
    ib, jb, rb = tensors.pair_list_bruteforce(pos, s.cell, rc, targets=targets)
    kb, vb = _keyed(ib, jb, rb, s.n)
    kk, vk = _keyed(i[keep], j[keep], r[keep], s.n)
    assert np.array_equal(kb, kk)
    assert np.abs(vb - vk).max() <= 1e-14 * float(s.cell[0, 0])
    # directed pairs come in (i, j), (j, i) couples with opposite vectors
    assert len(i) % 2 == 0
    fwd = dict(zip((i * s.n + j).tolist(), range(len(i))))
    for t in range(0, len(i), 9973):
        back = fwd[int(j[t]) * s.n + int(i[t])]
        assert torch.equal(r[back], -r[t])


def test_kdtree_pair_list_just_under_half_box():
    """Cutoff just under L/2 in the 10 A fluid: the k-d tree branch with the widest
    minimum-image shifts it can take."""
    s = synth.tiny_random(seed=1)
    L = s.cell[0, 0]
    rc = 0.5 * L * (1.0 - 1e-9)
    pos = torch.as_tensor(s.pos) + 3.0 * L      # positions in a far periodic image
    _compare_pair_lists(pos, s.cell, rc, None)
    _compare_pair_lists(pos, s.cell, rc, np.array([0, 5, 17, 95]))


# --- general cells ----------------------------------------------------------------

@pytest.fixture(scope="module")
def tri():
    return synth.triclinic_random()


@pytest.fixture(scope="module")
def tri_T(tri):
    return exact.tpbc_dense(tri.pos, tri.cell, 0.35 * synth.BOHR_ANGSTROM, tri.rvdw, BETA, DAMP)


def test_triclinic_tau_independence(tri, tri_T):
    for t in (0.25, 0.50):
        T = exact.tpbc_dense(tri.pos, tri.cell, t * synth.BOHR_ANGSTROM, tri.rvdw, BETA, DAMP)
        assert float((T - tri_T).norm() / tri_T.norm()) < 1e-12


def test_triclinic_block_trace_is_minus_four_pi_over_volume(tri, tri_T):
    N = tri.n
    V = abs(np.linalg.det(tri.cell))
    tr = tri_T.reshape(N, 3, N, 3).diagonal(dim1=1, dim2=3).sum(-1)
    assert float((tr + 4 * math.pi / V).abs().max()) < 1e-12 * 4 * math.pi / V


def test_same_lattice_in_a_skewed_basis():
    """A cubic lattice described by the right-handed basis (a1, a1 + a2, a3 + a1) is the
    same periodic system, so T^pbc must not change; the skewed description runs through
    the general-cell reciprocal vectors and image ranges."""
    s = synth.tiny_random(seed=2, n=24, L_ang=8.0, dmin_ang=1.8, sweeps=50)
    a1, a2, a3 = s.cell
    skew = np.array([a1, a1 + a2, a3 + a1])
    assert np.linalg.det(skew) > 0
    tau = 0.35 * synth.BOHR_ANGSTROM
    T0 = exact.tpbc_dense(s.pos, s.cell, tau, s.rvdw, BETA, DAMP)
    T1 = exact.tpbc_dense(s.pos, skew, tau, s.rvdw, BETA, DAMP)
    assert float((T1 - T0).norm() / T0.norm()) < 1e-12
    # the spherical real-space sum of the brute-force list is basis independent too
    rc = 13.0 * A
    i0, j0, r0 = tensors.pair_list_bruteforce(torch.as_tensor(s.pos), s.cell, rc)
    i1, j1, r1 = tensors.pair_list_bruteforce(torch.as_tensor(s.pos), skew, rc)
    assert len(i0) == len(i1)
    k0 = np.lexsort((r0[:, 2].numpy().round(9), r0[:, 1].numpy().round(9),
                     r0[:, 0].numpy().round(9), j0.numpy(), i0.numpy()))
    k1 = np.lexsort((r1[:, 2].numpy().round(9), r1[:, 1].numpy().round(9),
                     r1[:, 0].numpy().round(9), j1.numpy(), i1.numpy()))
    assert np.array_equal(i0.numpy()[k0], i1.numpy()[k1])
    assert np.array_equal(j0.numpy()[k0], j1.numpy()[k1])
    assert np.abs(r0.numpy()[k0] - r1.numpy()[k1]).max() < 1e-12


def test_triclinic_supercell(tri):
    """Doubling the skewed cell along a2: the field of a pattern repeated on both copies
    equals the field of the pattern in the original cell, on both copies."""
    tau = 0.35 * synth.BOHR_ANGSTROM
    a2 = tri.cell[1]
    sup = synth.System("tri2", np.concatenate([tri.pos, tri.pos + a2]),
                       np.array([tri.cell[0], 2 * a2, tri.cell[2]]),
                       np.tile(tri.alpha, 2), np.tile(tri.omega, 2), np.tile(tri.rvdw, 2))
    y = torch.randn(tri.n, 3, 2, dtype=torch.float64, generator=torch.Generator().manual_seed(4))
    want = exact.matvec_exact(tri, tau, BETA, DAMP, y)
    got = exact.matvec_exact(sup, tau, BETA, DAMP, torch.cat([y, y]))
    scale = float(want.abs().max())
    assert float((got[:tri.n] - want).abs().max()) < 1e-12 * scale
    assert float((got[tri.n:] - want).abs().max()) < 1e-12 * scale


def test_triclinic_matrix_free_matches_dense(tri, tri_T):
    tau = 0.35 * synth.BOHR_ANGSTROM
    C = exact.coupling_from_T(tri_T, tri.alpha, tri.omega)
    y = torch.randn(tri.n, 3, 2, dtype=torch.float64, generator=torch.Generator().manual_seed(6))
    want = (C @ y.reshape(-1, 2)).reshape(tri.n, 3, 2)
    got = exact.matvec_exact(tri, tau, BETA, DAMP, y)
    assert float((got - want).abs().max()) < 1e-13 * float(want.abs().max())


def test_triclinic_spme_converges_to_exact_ewald(tri):
    """SPME's reciprocal field on the skewed cell approaches the structure-factor sum
    monotonically in K, faster for higher spline order."""
    tau = 0.35 * synth.BOHR_ANGSTROM
    y = torch.randn(tri.n, 3, 2, dtype=torch.float64, generator=torch.Generator().manual_seed(8))
    want = exact.matvec_exact(tri, tau, BETA, DAMP, y, components=4)
    errs = []
    for K in (8, 12, 16, 24, 32):
        op = method.Operator(tri, method.MethodParams(tau=tau, r_pair=13 * A, grid=(K, K, K)))
        errs.append(float((op(y, method.REC) - want).abs().max() / want.abs().max()))
    assert all(e1 > e2 for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-6
    perr = []
    for p in (4, 6, 8):
        op = method.Operator(tri, method.MethodParams(tau=tau, r_pair=13 * A, grid=(16, 18, 20),
                                                      order=p))
        perr.append(float((op(y, method.REC) - want).abs().max() / want.abs().max()))
    assert perr[0] > perr[1] > perr[2], perr
    # and at a fine grid and high order the two agree closely
    g = torch.from_numpy(tri.omega * np.sqrt(tri.alpha))
    d = g[:, None, None] * y
    fine = spme.recip_field(torch.as_tensor(tri.pos), tri.cell, [40, 40, 40], 8, tau, d)
    assert float((g[:, None, None] * fine - want).abs().max() / want.abs().max()) < 1e-8
