"""Write the stored oracle values that the full-size GPU parity tests compare against.

Every number in the output comes from `oracle/` (plain CPU float64) applied to the
seeded synthetic workloads of `synth/`; nothing here calls or reads the GPU library.
The method parameters are derived with the oracle's own rules (oracle/params.py):
tau from erfc(tau r_c) / r_c = 1e-8 with r_c in Angstrom, r_pair = max(r_c, r_damp)
with 1 - f(r_damp) = 1e-4 at the largest damping radius, p = 6, and the workload's
grid (or the density rule of oracle/params.py when the workload gives none).

Outputs (numpy .npz, no pickles), one per workload:
  water24k_quadrature.npz   24,000-atom water box, K = 96, 50 Lanczos steps: per-probe
                            quadrature values Q_l for probes 0, 1, 62, 63, 64, 65, 126,
                            127 (both 64-wide grid chunks of the 128-probe block)
  organic12k_quadrature.npz 12,000-atom organic box, K = 80, 40 steps: probes 0 and 63
  uneven_quadrature.npz     batch of 32 water boxes, 40 steps: probe 0 of the smallest,
                            the median and the largest system
  water24k_rows.npz         C v of the 24k box for four seeded Gaussian right-hand sides
                            at 64 sampled atoms
Each file also stores the parameters it was computed with (tau, r_pair, grid, order,
seed, steps, probe indices, system index), which the tests check against the plan.

Run:  python tests/golden/make_oracle_goldens.py [name ...]   (minutes on 8 cores)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import lanczos as olz  # noqa: E402
from oracle import method as om  # noqa: E402
from oracle import params as opar  # noqa: E402

BETA, DAMP, DAMP_TOL, ORDER = 0.83, 6.0, 1e-4, 6


def derived(system, rc_ang, grid):
    """tau (1/bohr), r_pair (bohr) and the grid by the oracle's parameter rules."""
    tau = opar.tau_from_cutoff_angstrom(rc_ang) * synth.BOHR_ANGSTROM
    s_max = BETA * 2.0 * float(np.max(system.rvdw))
    r_pair = max(rc_ang * synth.ANGSTROM_BOHR, opar.damping_range(s_max, DAMP, DAMP_TOL))
    if grid is None:
        L = np.linalg.norm(system.cell, axis=1) * synth.BOHR_ANGSTROM
        grid = [opar.smooth_grid(x) for x in L]
    return tau, r_pair, [int(k) for k in grid]


def quadrature_golden(system, rc_ang, grid, seed, m, probes, sys_index=0):
    tau, r_pair, K = derived(system, rc_ang, grid)
    op = om.Operator(system, om.MethodParams(tau=tau, r_pair=r_pair, grid=tuple(K),
                                             order=ORDER, beta=BETA, d=DAMP))
    t0 = time.time()
    res = olz.slq(op, system.n, system.omega, seed=seed, n_probes=len(probes), m=m,
                  system=sys_index, reorth="none", probes=probes)
    print(f"  {system.n} atoms, K={K}, {len(probes)} probes x {m} steps: "
          f"{time.time() - t0:.0f} s", flush=True)
    return dict(q=res.q.detach().numpy(), probes=np.array(probes), tau=tau, r_pair=r_pair,
                grid=np.array(K), order=ORDER, seed=seed, steps=m, system=sys_index,
                n_atoms=system.n)


def water24k():
    wl = synth.workload("batched24k")
    return quadrature_golden(wl.systems[0], wl.real_cutoff_angstrom, [96] * 3, wl.probe_seed,
                             wl.n_steps, [0, 1, 62, 63, 64, 65, 126, 127])


def organic12k():
    wl = synth.workload("forces12k")
    return quadrature_golden(wl.systems[0], wl.real_cutoff_angstrom, [80] * 3, wl.probe_seed,
                             wl.n_steps, [0, 63])


def uneven():
    wl = synth.workload("uneven")
    sizes = [x.n for x in wl.systems]
    order = np.argsort(sizes, kind="stable")
    picks = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    out = {}
    for tag, k in zip(("smallest", "median", "largest"), picks):
        g = quadrature_golden(wl.systems[k], wl.real_cutoff_angstrom, None, wl.probe_seed,
                              wl.n_steps, [0], sys_index=k)
        for key, v in g.items():
            out[f"{tag}_{key}"] = v
    return out


def water24k_rows():
    """C v for four right-hand sides (columns 0, 63, 64, 127 of the seeded Gaussian block
    synth.gaussian_block(2024, 128, N)) at 64 sampled atoms (synth.sample_atoms(5, N)),
    through the oracle's method operator with the derived parameters."""
    wl = synth.workload("batched24k")
    s = wl.systems[0]
    tau, r_pair, K = derived(s, wl.real_cutoff_angstrom, [96] * 3)
    op = om.Operator(s, om.MethodParams(tau=tau, r_pair=r_pair, grid=tuple(K), order=ORDER,
                                        beta=BETA, d=DAMP))
    cols = [0, 63, 64, 127]
    v = synth.gaussian_block(2024, 128, s.n)[cols]
    sample = synth.sample_atoms(5, s.n)
    t0 = time.time()
    import torch
    out = op(torch.from_numpy(v).permute(1, 2, 0).contiguous()).permute(2, 0, 1)
    print(f"  rows: {time.time() - t0:.0f} s", flush=True)
    return dict(rows=out[:, sample].numpy(), columns=np.array(cols), sample=sample,
                block_seed=2024, block=128, tau=tau, r_pair=r_pair, grid=np.array(K),
                order=ORDER)


MAKERS = {"water24k_quadrature": water24k, "organic12k_quadrature": organic12k,
          "uneven_quadrature": uneven, "water24k_rows": water24k_rows}


def main(names):
    for name in names or MAKERS:
        print(name, flush=True)
        np.savez(os.path.join(HERE, name + ".npz"), **MAKERS[name]())


if __name__ == "__main__":
    main(sys.argv[1:])
