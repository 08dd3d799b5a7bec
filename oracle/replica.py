"""Replica method (oracle): truncated sum of damped tensors over periodic images.

Theory section, eq. replica and the replica figure: T^pbc_ij = T'_ij(j in 0) +
sum_{n != 0} T'_ij(j in n), images chosen by a spherical cutoff R_cut around
atom i inside the supercell of +-n_max cells. The sum is conditionally
convergent; with a spherical cutoff it tends to the vacuum (spherical)
boundary limit, which exceeds the tin-foil Ewald tensor by (4 pi / (3 V)) I_3
in every block.
"""
from __future__ import annotations

import torch

from . import tensors as tz


def replica_field(sys, beta, d, rcut, dvec):
    """sum over (j, n) with |R_j + n - R_i| < rcut of f T d_j; dvec (N, 3, B)."""
    pos = torch.as_tensor(sys.pos, dtype=torch.float64)
    rvdw = torch.as_tensor(sys.rvdw, dtype=torch.float64)
    N = pos.shape[0]
    i, j, r = tz.pair_list_bruteforce(pos, sys.cell, rcut)
    rn = torch.sqrt((r * r).sum(-1))
    A, B = tz.radial_damped(rn, beta * (rvdw[i] + rvdw[j]), d)
    out = torch.zeros_like(dvec)
    return out.index_add(0, i, tz.apply_pairs(A, B, r, dvec[j]))
