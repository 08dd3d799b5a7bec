"""The direct-space cutoff reading (the damping tail outlives the erfc cutoff; the
library runs its pair kernel to r_pair = max(r_c, r_damp) with 1 - f(r_damp) = 1e-4 at
the largest damping radius, which is r_c = 9 A on the 24,000-atom water box).

This measures, on sampled rows of that box, what the cutoff leaves out: the direct
field between 9 A and a converged cutoff (tau r >= 6 and r >= 7.2 S_max, where
1 - f < 1e-16), against the size of C v and against the SPME discretization error of
the same box (K = 96, p = 6) relative to the exact Ewald sum. The tail must stay well
below both 1e-6 of max |C v| and the discretization error."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import exact, method, params, tensors

A = synth.ANGSTROM_BOHR
BETA, DAMP = 0.83, 6.0


@pytest.mark.slow
def test_pair_cutoff_tail_on_the_24k_water_box():
    s = synth.water_box(8000, seed=3)
    tau = params.tau_from_cutoff_angstrom(9.0) * synth.BOHR_ANGSTROM
    S = BETA * 2 * float(s.rvdw.max())
    r_pair = max(9.0 * A, params.damping_range(S, DAMP, 1e-4))
    assert r_pair == 9.0 * A
    r_conv = max(6.0 / tau, 7.2 * S)
    pos = torch.as_tensor(s.pos)
    rng = np.random.default_rng(0)
    targets = np.sort(rng.choice(s.n, 64, replace=False))
    tt = torch.from_numpy(targets)
    g = torch.from_numpy(s.omega * np.sqrt(s.alpha))
    y = torch.from_numpy(rng.choice([-1.0, 1.0], size=(s.n, 3, 2)) / math.sqrt(3 * s.n))
    d = g[:, None, None] * y
    rv = torch.from_numpy(s.rvdw)
    loc = torch.full((s.n,), -1, dtype=torch.long)
    loc[tt] = torch.arange(len(targets))

    def e_dir(rc):
        i, j, r = tensors.pair_list(pos, s.cell, rc, targets=targets)
        rn = torch.sqrt((r * r).sum(-1))
        a, b = tensors.radial_direct(rn, tau, BETA * (rv[i] + rv[j]), DAMP)
        out = torch.zeros(len(targets), 3, 2, dtype=torch.float64)
        return out.index_add(0, loc[i], tensors.apply_pairs(a, b, r, d[j]))

    tail = g[tt][:, None, None] * (e_dir(r_conv) - e_dir(r_pair))
    op = method.Operator(s, method.MethodParams(tau=tau, r_pair=r_pair, grid=(96, 96, 96)))
    Cv = op(y)[tt]
    rec_err = op(y, method.REC)[tt] - exact.matvec_exact(s, tau, BETA, DAMP, y, targets=targets,
                                                         components=4)
    scale = float(Cv.abs().max())
    tail_rel = float(tail.abs().max()) / scale
    disc_rel = float(rec_err.abs().max()) / scale
    print(f"direct tail beyond 9 A: {tail_rel:.2e} of max|Cv|; "
          f"SPME(K=96, p=6) vs exact Ewald: {disc_rel:.2e}")
    assert tail_rel < 1e-6
    assert tail_rel < 0.1 * disc_rel
