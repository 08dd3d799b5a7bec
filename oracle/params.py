"""Parameter rules (oracle copy).

- Ewald tau: the paper fixes tau = 0.544590 for a 7 Angstrom real-space
  cutoff (end of the Theory section) without stating the rule. The rule used
  here, erfc(tau r_c) / r_c = 1e-8 with r_c in Angstrom and tau in 1/Angstrom,
  reproduces that number (pinned in the tests).
- Damping range: 1 - f(r) of the Fermi damping falls below a tolerance at
  r_damp = S (1 + ln(1/tol - 1) / d), with S = beta (R_i + R_j).
- Grid: the paper's default density is 1.2 points per Angstrom per box edge
  (Numerical results). The workloads here use the smallest even 2^a 3^b that
  is >= 1.4 points per Angstrom when no grid is given.
"""
from __future__ import annotations

import math

from scipy.special import erfc

BOHR_ANGSTROM = 0.529177210903


def tau_from_cutoff_angstrom(rc_ang: float, eps: float = 1e-8) -> float:
    """Solve erfc(tau rc) / rc = eps for tau by bisection; rc and 1/tau in Angstrom."""
    lo, hi = 0.0, 1.0
    while erfc(hi * rc_ang) / rc_ang > eps:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if erfc(mid * rc_ang) / rc_ang > eps:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def damping_range(s_max: float, d: float, tol: float) -> float:
    """Distance where 1 - f = tol for the largest damping radius s_max."""
    return s_max * (1.0 + math.log(1.0 / tol - 1.0) / d)


def smooth_grid(length_ang: float, density: float = 1.4) -> int:
    """Smallest even 2^a 3^b >= density * length."""
    target = density * length_ang
    best = None
    a = 1
    while 2 ** a <= 4 * target + 8:
        b = 0
        while 2 ** a * 3 ** b <= 4 * target + 8:
            k = 2 ** a * 3 ** b
            if k >= target and (best is None or k < best):
                best = k
            b += 1
        a += 1
    return best
