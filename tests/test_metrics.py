"""Interval estimates used by the long-run statistical parity and the bench.

Newcombe's hybrid score interval is pinned to the published worked examples
(tests/golden/newcombe_cases.json, four decimals); Welch's interval to
scipy's own Welch test and to its coverage on samples of equal means.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2203_08361_amd import metrics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "newcombe_cases.json")


def test_newcombe_published_examples():
    cases = json.load(open(GOLDEN))["cases"]
    for c in cases:
        lo, hi = metrics.newcombe_interval(c["k1"], c["n1"], c["k2"], c["n2"])
        assert lo == pytest.approx(c["lower"], abs=6e-5)
        assert hi == pytest.approx(c["upper"], abs=6e-5)


def test_newcombe_symmetry_and_point_estimate():
    for k1, n1, k2, n2 in [(3, 40, 7, 50), (0, 30, 0, 30), (30, 30, 12, 31)]:
        lo, hi = metrics.newcombe_interval(k1, n1, k2, n2)
        lo2, hi2 = metrics.newcombe_interval(k2, n2, k1, n1)
        assert lo == pytest.approx(-hi2, abs=1e-15) and hi == pytest.approx(-lo2, abs=1e-15)
        assert lo <= k1 / n1 - k2 / n2 <= hi


def test_welch_matches_scipy():
    from scipy import stats

    rng = np.random.default_rng(5)
    for na, nb, sa, sb in [(20, 30, 1.0, 3.0), (200, 150, 2.0, 0.5), (5, 7, 1.0, 1.0)]:
        a = rng.normal(0.3, sa, na)
        b = rng.normal(0.0, sb, nb)
        lo, hi = metrics.welch_interval(a, b)
        ci = stats.ttest_ind(a, b, equal_var=False).confidence_interval(0.95)
        assert lo == pytest.approx(ci.low, rel=1e-10) and hi == pytest.approx(ci.high, rel=1e-10)


def test_welch_coverage_with_equal_means():
    rng = np.random.default_rng(11)
    hits = 0
    trials = 2000
    for _ in range(trials):
        a = rng.normal(1.0, 1.0, 25)
        b = rng.normal(1.0, 2.5, 40)
        lo, hi = metrics.welch_interval(a, b)
        hits += lo <= 0.0 <= hi
    assert 0.93 <= hits / trials <= 0.97


def test_wilson_ends_and_step_to_solution_of_tiny_P():
    for n in (1, 4, 24, 128, 1024, 10**4):
        assert metrics.wilson_interval(0, n)[0] == 0.0
        assert metrics.wilson_interval(n, n)[1] == 1.0
        if n > 1:
            lo, hi = metrics.wilson_interval(1, n)
            assert 0.0 < lo < 1.0 / n < hi
    # eq. (15) stays finite and decreasing for P far below the rounding of 1 - P
    S = [metrics.step_to_solution(P, 100) for P in (1e-3, 1e-12, 1e-17, 1e-300)]
    assert all(math.isfinite(x) for x in S) and S == sorted(S)
    assert S[2] == pytest.approx(100 * math.log(100) / 1e-17, rel=1e-12)
