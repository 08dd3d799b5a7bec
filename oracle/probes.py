"""Rademacher probe vectors (eq. dds) from a counter-based SplitMix64 stream.

The Hutchinson estimator (eq. hutch) uses R vectors v_l = u_l / ||u_l|| with
entries u_{l,i} = +-1 at probability 1/2; for D = 3N entries ||u_l|| = sqrt(D).

The signs are drawn from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014):
output number n (0-based) of the stream seeded with s is mix(s + (n+1) G)
modulo 2^64, with G = 0x9E3779B97F4A7C15 and the mix function
z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB;
z ^= z >> 31. This module implements it independently of the GPU library.

Key layout (shared definition, separate implementations):
  system seed  z_s = output s of the stream seeded with `seed`
  entry (l, i, alpha) of system s: sign from output (l * 3N + 3 i + alpha)
  of the stream seeded with z_s; the sign is -1 when bit 63 is set.
  i is the atom's index in the caller's (original) order.
"""
from __future__ import annotations

import numpy as np
import torch

_G = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, index) -> np.ndarray:
    """Outputs number `index` (array, 0-based) of the stream seeded with `seed`."""
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed % (1 << 64)) + (idx + np.uint64(1)) * _G
    return _mix(z)


def system_seed(seed: int, system: int) -> int:
    return int(splitmix64(seed, np.array([system]))[0])


def rademacher(seed: int, system: int, n_atoms: int, probes) -> torch.Tensor:
    """Probe block v[l, i, alpha] = +-1/sqrt(3N) for the given probe indices l."""
    probes = np.asarray(list(probes), dtype=np.uint64)
    zs = system_seed(seed, system)
    D = 3 * n_atoms
    idx = probes[:, None] * np.uint64(D) + np.arange(D, dtype=np.uint64)[None, :]
    bits = splitmix64(zs, idx) >> np.uint64(63)
    signs = 1.0 - 2.0 * bits.astype(np.float64)
    return torch.from_numpy(signs.reshape(len(probes), n_atoms, 3) / np.sqrt(D))
