"""Seeded synthetic periodic systems in atomic units (bohr, bohr^3, Hartree).

The paper's own test systems (a 216-molecule water box of 18.64 Angstrom and
a 14.2 Angstrom diamond box, Numerical results section) and their
atom-in-molecule parameters are not published, so these generators build
stand-ins with the same structure: liquid water at 1 g/cm^3, a dense random
fluid, an organic-like random solid, and diamond.

Nothing in this module evaluates the MBD method; it only places atoms and
assigns the per-atom inputs (alpha, omega, R_vdW) that the MBD Hamiltonian
takes (Review of the MBD section, eq. ham).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# CODATA 2018 Bohr radius in Angstrom.
BOHR_ANGSTROM = 0.529177210903
ANGSTROM_BOHR = 1.0 / BOHR_ANGSTROM

# Liquid water at 1 g/cm^3: N_A / 18.01528 g/mol per cm^3, in molecules / A^3.
WATER_NUMBER_DENSITY = 6.02214076e23 / 18.01528 * 1e-24


@dataclass
class System:
    """One periodic system. Positions in bohr; cell rows are a1, a2, a3 in bohr."""
    name: str
    pos: np.ndarray          # (N, 3) float64, bohr
    cell: np.ndarray         # (3, 3) float64, rows = lattice vectors, bohr
    alpha: np.ndarray        # (N,) bohr^3
    omega: np.ndarray        # (N,) Hartree
    rvdw: np.ndarray         # (N,) bohr

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


@dataclass
class Workload:
    """A system (or batch of systems) plus the method settings it is run with.

    tau_inv_angstrom None means: derive it from the real-space cutoff.
    grid None (per system) means: derive it from the grid-density rule.
    """
    name: str
    systems: List[System]
    beta: float = 0.83
    damp_d: float = 6.0
    tau_inv_angstrom: Optional[float] = None
    real_cutoff_angstrom: float = 9.0
    grid: Optional[List[Optional[int]]] = None
    spline_order: int = 6
    n_probes: int = 8
    n_steps: int = 30
    block: int = 1
    precision: str = "fp64"          # "fp64" or "mixed"
    want_forces: bool = False
    probe_seed: int = 12345
    notes: str = ""
    extra: dict = field(default_factory=dict)


def _cubic(L_bohr: float) -> np.ndarray:
    return np.eye(3) * L_bohr


def _min_image(dx: np.ndarray, L: float) -> np.ndarray:
    return dx - L * np.round(dx / L)


def tiny_random(seed: int = 1, n: int = 96, L_ang: float = 10.0,
                dmin_ang: float = 2.0, sweeps: int = 500) -> System:
    """Dense random fluid: n atoms in a cubic box with a hard-core minimum distance.

    The packing fraction (pi/6) dmin^3 n / L^3 = 0.40 is above the random
    sequential adsorption limit, so the recipe starts from random sites of a
    simple-cubic lattice of spacing dmin and equilibrates with hard-sphere
    Metropolis moves (max step 0.1 dmin, minimum image).
    """
    rng = np.random.default_rng(seed)
    m = int(round(L_ang / dmin_ang))
    sites = np.array([(i, j, k) for i in range(m) for j in range(m) for k in range(m)], float)
    sites = (sites + 0.5) * (L_ang / m)
    pos = sites[rng.choice(len(sites), n, replace=False)].copy()
    step = 0.1 * dmin_ang
    d2min = dmin_ang * dmin_ang
    for _ in range(sweeps):
        for a in rng.permutation(n):
            trial = (pos[a] + rng.uniform(-step, step, 3)) % L_ang
            dx = _min_image(pos - trial, L_ang)
            r2 = np.einsum("ij,ij->i", dx, dx)
            r2[a] = np.inf
            if r2.min() >= d2min:
                pos[a] = trial
    return System(
        name=f"tiny_random_n{n}",
        pos=pos * ANGSTROM_BOHR,
        cell=_cubic(L_ang * ANGSTROM_BOHR),
        alpha=rng.uniform(5.0, 15.0, n),
        omega=rng.uniform(0.3, 0.7, n),
        rvdw=rng.uniform(3.0, 4.0, n),
    )


class _RSA:
    """Periodic bucket grid for random sequential addition in a cubic box."""

    def __init__(self, L: float, n_atoms: int, reach: float, slots: int = 32):
        self.L = L
        self.nc = max(1, int(L // reach))
        self.h = L / self.nc
        self.occ = np.full((self.nc, self.nc, self.nc, slots), -1, np.int64)
        self.fill = np.zeros((self.nc, self.nc, self.nc), np.int64)
        self.P = np.zeros((n_atoms, 3))
        self.T = np.zeros(n_atoms, np.int64)
        self.count = 0
        span = np.arange(-1, 2) if self.nc >= 3 else np.arange(self.nc)
        self.offsets = np.array([(a, b, c) for a in span for b in span for c in span])

    def neighbours(self, centres):
        c = np.floor(centres / self.h).astype(np.int64) % self.nc
        cells = (c[:, None, :] + self.offsets[None, :, :]) % self.nc
        kmax = max(1, int(self.fill.max()))
        idx = self.occ[cells[..., 0], cells[..., 1], cells[..., 2], :kmax]
        return idx.reshape(len(centres), -1)

    def insert(self, atoms, types):
        for a, t in zip(atoms, types):
            c = tuple(np.floor(a / self.h).astype(np.int64) % self.nc)
            k = self.fill[c]
            if k >= self.occ.shape[3]:
                raise RuntimeError("random addition: bucket overflow")
            self.occ[c + (k,)] = self.count
            self.fill[c] = k + 1
            self.P[self.count] = a
            self.T[self.count] = t
            self.count += 1


def _rsa_fill(L, n_units, unit_types, sample_units, min_dist, reach, rng, batch=1024):
    """Random sequential addition of n_units rigid units (one or more atoms).

    Candidates come in vectorized batches and are tested against the atoms
    already placed; survivors are accepted in proposal order after a check
    against units accepted earlier in the same batch, which is the same as
    one-at-a-time addition over the same proposal stream.
    min_dist[t_new][t_old] is the hard-core distance between atom types;
    reach must be at least the largest hard core plus the unit radius.
    """
    types = np.asarray(unit_types)
    na = len(types)
    rsa = _RSA(L, n_units * na, reach)
    md2 = np.asarray(min_dist, float) ** 2
    placed = 0
    stall = 0
    while placed < n_units:
        atoms = sample_units(batch) % L                      # (M, na, 3)
        nb = rsa.neighbours(atoms[:, 0, :])                  # (M, K)
        valid = nb >= 0
        safe = np.where(valid, nb, 0)
        near = rsa.P[safe]                                   # (M, K, 3)
        tnear = rsa.T[safe]
        # Stage 1: the unit's first atom only (cheap, rejects most proposals).
        d = atoms[:, 0, None, :] - near
        d -= L * np.round(d / L)
        r2 = np.einsum("mkc,mkc->mk", d, d)
        clash = ((r2 < md2[types[0], tnear]) & valid).any(axis=1)
        keep = np.nonzero(~clash)[0]
        # Stage 2: every atom of the surviving units.
        if na > 1 and keep.size:
            d = atoms[keep][:, :, None, :] - near[keep][:, None, :, :]
            d -= L * np.round(d / L)
            r2 = np.einsum("makc,makc->mak", d, d)
            lim = md2[types[None, :, None], tnear[keep][:, None, :]]
            clash[keep] = ((r2 < lim) & valid[keep][:, None, :]).any(axis=(1, 2))
        accepted = []
        start = rsa.count
        for m in np.nonzero(~clash)[0]:
            if rsa.count > start:
                nb = rsa.neighbours(atoms[m, :1, :])[0]
                nb = nb[nb >= start]
                if nb.size:
                    d = atoms[m][:, None, :] - rsa.P[nb][None, :, :]
                    d -= L * np.round(d / L)
                    r2 = np.einsum("akc,akc->ak", d, d)
                    if (r2 < md2[types[:, None], rsa.T[nb][None, :]]).any():
                        continue
            rsa.insert(atoms[m], types)
            accepted.append(m)
            if placed + len(accepted) == n_units:
                break
        placed += len(accepted)
        stall = stall + 1 if not accepted else 0
        if stall > 500:
            raise RuntimeError("random sequential addition stalled")
    return rsa.P


def water_box(n_mol: int, seed: int, oo_min_ang: float = 2.5,
              inter_min_ang: float = 1.5) -> System:
    """Rigid water molecules at 1 g/cm^3 (O-H 0.96 A, H-O-H 104.5 deg).

    Random sequential addition of molecules with O-O >= 2.5 A, a random
    orientation per molecule (normalized 4-Gaussian quaternion), and rejection
    of any other intermolecular atom pair closer than 1.5 A.
    Parameters: alpha_O = 7, alpha_H = 2.5 bohr^3; omega_O = 0.6,
    omega_H = 0.45 Ha; R_vdW,O = 3.6, R_vdW,H = 3.1 bohr.
    Atom order is O, H, H per molecule.
    """
    rng = np.random.default_rng(seed)
    L = (n_mol / WATER_NUMBER_DENSITY) ** (1.0 / 3.0)
    roh, ang = 0.96, math.radians(104.5)
    local = np.array([[0.0, 0.0, 0.0],
                      [roh * math.sin(ang / 2), 0.0, roh * math.cos(ang / 2)],
                      [-roh * math.sin(ang / 2), 0.0, roh * math.cos(ang / 2)]])

    def sample(m):
        o = rng.uniform(0.0, L, (m, 3))
        q = rng.normal(size=(m, 4))
        q /= np.linalg.norm(q, axis=1, keepdims=True)
        w, x, y, z = q.T
        R = np.stack([
            np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
            np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
            np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1),
        ], 1)
        return o[:, None, :] + np.einsum("mij,aj->mai", R, local)

    md = [[oo_min_ang, inter_min_ang], [inter_min_ang, inter_min_ang]]
    pos = _rsa_fill(L, n_mol, [0, 1, 1], sample, md, oo_min_ang + 2 * roh, rng)
    n = pos.shape[0]
    is_o = np.zeros(n, bool)
    is_o[0::3] = True
    return System(
        name=f"water_{n_mol}",
        pos=pos * ANGSTROM_BOHR,
        cell=_cubic(L * ANGSTROM_BOHR),
        alpha=np.where(is_o, 7.0, 2.5),
        omega=np.where(is_o, 0.6, 0.45),
        rvdw=np.where(is_o, 3.6, 3.1),
    )


def organic_mix(seed: int = 4, n: int = 12000, L_ang: float = 50.0,
                dmin_ang: float = 1.1) -> System:
    """Random organic-like solid: 60 % C, 30 % H, 10 % O with exact counts.

    C: alpha 12, omega 0.45; H: alpha 4.5, omega 0.4; O: alpha 5.4, omega 0.55
    (bohr^3, Ha). R_vdW uses free-atom radii C 3.59, H 3.10, O 3.19 bohr.
    Random sequential addition with a 1.1 A minimum distance.
    """
    rng = np.random.default_rng(seed)
    nC, nH = int(round(0.6 * n)), int(round(0.3 * n))
    nO = n - nC - nH
    kind = np.array([0] * nC + [1] * nH + [2] * nO)
    rng.shuffle(kind)
    pos = _rsa_fill(L_ang, n, [0], lambda m: rng.uniform(0.0, L_ang, (m, 1, 3)),
                    [[dmin_ang]], dmin_ang, rng)
    alpha = np.array([12.0, 4.5, 5.4])[kind]
    omega = np.array([0.45, 0.4, 0.55])[kind]
    rvdw = np.array([3.59, 3.10, 3.19])[kind]
    return System(name=f"organic_{n}", pos=pos * ANGSTROM_BOHR,
                  cell=_cubic(L_ang * ANGSTROM_BOHR), alpha=alpha, omega=omega, rvdw=rvdw)


def uneven_water_batch(seed: int = 5, count: int = 32, n_lo: int = 500,
                       n_hi: int = 20000) -> List[System]:
    """Water boxes with atom counts log-uniform in [n_lo, n_hi] (multiples of 3)."""
    out = []
    for s in range(count):
        rng = np.random.default_rng(5000 + s)
        n_atoms = 3 * int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi))) / 3.0))
        out.append(water_box(n_atoms // 3, seed=5000 + s))
    return out


def one_atom(alpha: float = 10.0, omega: float = 0.5, rvdw: float = 3.5,
             L_ang: float = 10.0, at=(0.0, 0.0, 0.0)) -> System:
    L = L_ang * ANGSTROM_BOHR
    return System("one_atom", np.array([at], float) * ANGSTROM_BOHR, _cubic(L),
                  np.array([alpha]), np.array([omega]), np.array([rvdw]))


def simple_cubic(n_side: int, a_ang: float, alpha: float = 8.0, omega: float = 0.5,
                 rvdw: float = 3.3) -> System:
    idx = np.array([(i, j, k) for i in range(n_side) for j in range(n_side)
                    for k in range(n_side)], float)
    n = idx.shape[0]
    return System(f"sc_{n_side}", idx * a_ang * ANGSTROM_BOHR,
                  _cubic(n_side * a_ang * ANGSTROM_BOHR),
                  np.full(n, alpha), np.full(n, omega), np.full(n, rvdw))


def dimer(r_ang: float, L_ang: float = 200.0, alpha: float = 10.0, omega: float = 0.5,
          rvdw: float = 3.5) -> System:
    c = 0.5 * L_ang
    pos = np.array([[c - 0.5 * r_ang, c, c], [c + 0.5 * r_ang, c, c]]) * ANGSTROM_BOHR
    return System("dimer", pos, _cubic(L_ang * ANGSTROM_BOHR), np.full(2, alpha),
                  np.full(2, omega), np.full(2, rvdw))


def diamond_box(n_cells: int = 4, a_ang: float = 3.567) -> System:
    """Diamond: n_cells^3 conventional cubic cells (8 atoms each), carbon parameters."""
    base = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0],
                     [.25, .25, .25], [.25, .75, .75], [.75, .25, .75], [.75, .75, .25]])
    pts = []
    for i in range(n_cells):
        for j in range(n_cells):
            for k in range(n_cells):
                pts.append(base + np.array([i, j, k]))
    pos = np.concatenate(pts) * a_ang
    n = pos.shape[0]
    return System(f"diamond_{n_cells}", pos * ANGSTROM_BOHR,
                  _cubic(n_cells * a_ang * ANGSTROM_BOHR), np.full(n, 12.0),
                  np.full(n, 0.45), np.full(n, 3.59))


def gaussian_block(seed: int, nrhs: int, n_atoms: int) -> np.ndarray:
    """Seeded standard-normal test vectors [nrhs][n_atoms][3] (numpy PCG64)."""
    return np.random.default_rng(seed).standard_normal((nrhs, n_atoms, 3))


def sample_atoms(seed: int, n_atoms: int, count: int = 64) -> np.ndarray:
    """A seeded sorted sample of distinct atom indices."""
    return np.sort(np.random.default_rng(seed).choice(n_atoms, min(count, n_atoms),
                                                      replace=False))


# A skewed right-handed cell (rows a1, a2, a3 in Angstrom) for the general-cell cases.
SKEWED_CELL_ANGSTROM = np.array([[10.0, 0.0, 0.0], [2.6, 9.4, 0.0], [-1.7, 2.1, 10.8]])


def triclinic_random(n: int = 80, seed: int = 3, dmin_ang: float = 1.6,
                     cell_ang: Optional[np.ndarray] = None) -> System:
    """Random atoms in a triclinic cell (default: SKEWED_CELL_ANGSTROM) with a minimum
    periodic-image distance dmin, by rejection on uniform fractional coordinates;
    alpha ~ U[5, 15], omega ~ U[0.3, 0.7], R_vdW ~ U[3, 4] as in the dense fluid."""
    cell = SKEWED_CELL_ANGSTROM if cell_ang is None else np.asarray(cell_ang, float)
    rng = np.random.default_rng(seed)
    shifts = np.array([[i, j, k] for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)])
    pts = []
    while len(pts) < n:
        f = rng.uniform(0.0, 1.0, 3)
        ok = True
        for q in pts:
            d = (f - q)[None, :] + shifts
            if np.min(np.linalg.norm(d @ cell, axis=1)) < dmin_ang:
                ok = False
                break
        if ok:
            pts.append(f)
    pos = np.array(pts) @ cell
    alpha = rng.uniform(5.0, 15.0, n)
    omega = rng.uniform(0.3, 0.7, n)
    rvdw = rng.uniform(3.0, 4.0, n)
    return System("triclinic", pos * ANGSTROM_BOHR, cell * ANGSTROM_BOHR, alpha, omega, rvdw)


def workload(name: str) -> Workload:
    """The five synthetic workloads (tiny, medium, batched 24k, forces 12k, uneven).

    Grid sizes given explicitly follow the workload definitions; None means the
    grid-density rule picks them.
    """
    if name == "tiny":
        s = tiny_random(seed=1)
        return Workload("tiny", [s], tau_inv_angstrom=0.35, real_cutoff_angstrom=13.0,
                        grid=[16], n_probes=8, n_steps=30, block=1, precision="fp64",
                        notes="N=96 hard-sphere fluid, L=10 A; stated 5 A real cutoff is "
                              "run at 13 A so that erfc truncation stays below 1e-9")
    if name == "medium":
        s = water_box(1000, seed=2)
        return Workload("medium", [s], tau_inv_angstrom=None, real_cutoff_angstrom=7.0,
                        grid=[48], n_probes=32, n_steps=40, block=1, precision="fp64")
    if name == "batched24k":
        s = water_box(8000, seed=3)
        return Workload("batched24k", [s], tau_inv_angstrom=None, real_cutoff_angstrom=9.0,
                        grid=[96], n_probes=128, n_steps=50, block=128, precision="mixed")
    if name == "forces12k":
        s = organic_mix(seed=4)
        return Workload("forces12k", [s], tau_inv_angstrom=None, real_cutoff_angstrom=9.0,
                        grid=[80], n_probes=64, n_steps=40, block=64, precision="mixed",
                        want_forces=True)
    if name == "uneven":
        systems = uneven_water_batch(seed=5)
        return Workload("uneven", systems, tau_inv_angstrom=None, real_cutoff_angstrom=9.0,
                        grid=None, n_probes=64, n_steps=40, block=64, precision="mixed",
                        want_forces=True)
    raise KeyError(name)
