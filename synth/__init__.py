"""Seeded synthetic inputs shared by the oracle and the GPU library's tests/bench.

This package only generates input arrays (positions, cell, atomic parameters)
and the per-workload method settings. It contains none of the method's
arithmetic: no tensors, no Ewald sums, no splines, no Lanczos.
"""
from .systems import (  # noqa: F401
    BOHR_ANGSTROM, ANGSTROM_BOHR, System, Workload,
    tiny_random, water_box, organic_mix, uneven_water_batch,
    one_atom, simple_cubic, dimer, diamond_box, workload,
    SKEWED_CELL_ANGSTROM, triclinic_random, gaussian_block, sample_atoms,
)
