"""Evaluation quantities of the paper computed from library outputs.

These are host-side statistics over replicas (not part of the per-step path):
  - cut value, eq. (14): C = -E/2 - (1/4) sum_ij J_ij  (MAX-CUT with w = -J)
  - success probability P: fraction of trials reaching the target energy
    (Results, K2000 statistics)
  - step-to-solution, eq. (15): S = Ns log(0.01) / log(1 - P); time-to-solution
    is S times the time per step.
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
    return (max(0.0, c - h), min(1.0, c + h))


def step_to_solution(P: float, Ns: int) -> float:
    """Eq. (15); infinite when P = 0, Ns when P >= 0.99 (one run suffices)."""
    if P <= 0.0:
        return math.inf
    if P >= 0.99:
        return float(Ns)
    return Ns * math.log(0.01) / math.log(1.0 - P)
