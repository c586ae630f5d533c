"""Evaluation quantities of the paper computed from library outputs.

These are host-side statistics over replicas (not part of the per-step path):
  - cut value, eq. (14): C = -E/2 - (1/4) sum_ij J_ij  (MAX-CUT with w = -J)
  - success probability P: fraction of trials reaching the target energy
    (Results, K2000 statistics)
  - step-to-solution, eq. (15): S = Ns log(0.01) / log(1 - P); time-to-solution
    is S times the time per step;
  - interval estimates for comparing two sets of runs: Wilson for a
    proportion, Newcombe's hybrid score interval for a difference of two
    proportions, Welch's t interval for a difference of two means.
"""
from __future__ import annotations

import math

import numpy as np


def cut_from_energy(E, J) -> np.ndarray:
    """Eq. (14)."""
    return -0.5 * np.asarray(E, dtype=np.float64) - 0.25 * float(np.asarray(J, np.float64).sum())


def success_probability(E, target: float) -> float:
    E = np.asarray(E, dtype=np.float64)
    return float(np.mean(E <= target)) if E.size else 0.0


def wilson_interval(k: int, n: int, z: float = 1.959963984540054):
    """95% Wilson score interval of a binomial proportion k/n."""
    if n <= 0:
        return (0.0, 1.0)
    p = k / n
    den = 1 + z * z / n
    c = (p + z * z / (2 * n)) / den
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / den
    # the ends are exactly 0 at k = 0 and 1 at k = n (c - h, c + h round near them)
    lo = 0.0 if k == 0 else max(0.0, c - h)
    hi = 1.0 if k == n else min(1.0, c + h)
    return (lo, hi)


def step_to_solution(P: float, Ns: int) -> float:
    """Eq. (15); infinite when P = 0, Ns when P >= 0.99 (one run suffices)."""
    if P <= 0.0:
        return math.inf
    if P >= 0.99:
        return float(Ns)
    q = 1.0 - P
    # a P below the rounding of 1 - P: log1p keeps S finite (and very large)
    return Ns * math.log(0.01) / (math.log(q) if q < 1.0 else math.log1p(-P))


def newcombe_interval(k1: int, n1: int, k2: int, n2: int, z: float = 1.959963984540054):
    """95% interval for p1 - p2 (p = k/n) from the two Wilson intervals
    (Newcombe's hybrid score method, no continuity correction)."""
    l1, u1 = wilson_interval(k1, n1, z)
    l2, u2 = wilson_interval(k2, n2, z)
    p1, p2 = k1 / n1, k2 / n2
    d = p1 - p2
    return (d - math.sqrt((p1 - l1) ** 2 + (u2 - p2) ** 2),
            d + math.sqrt((u1 - p1) ** 2 + (p2 - l2) ** 2))


def welch_interval(a, b, level: float = 0.95):
    """Interval for mean(a) - mean(b) with unequal variances (Welch's t with the
    Welch-Satterthwaite degrees of freedom)."""
    from scipy import stats

    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    va, vb = a.var(ddof=1) / a.size, b.var(ddof=1) / b.size
    d = a.mean() - b.mean()
    se = math.sqrt(va + vb)
    if se == 0.0:
        return (d, d)
    df = (va + vb) ** 2 / (va * va / (a.size - 1) + vb * vb / (b.size - 1))
    t = stats.t.ppf(0.5 + level / 2, df)
    return (d - t * se, d + t * se)
