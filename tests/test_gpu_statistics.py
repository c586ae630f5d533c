"""Long-run statistical parity of bSB (marked `gpu`).

A long bSB trajectory is chaotic, so it is compared with the FP64 oracle in
distribution rather than pointwise: over R = 256 replicas of short runs on
N = 300 instances (300 steps for SK, 400 for Gaussian couplings: short enough
that the best energies still spread over many values instead of all replicas
reaching one optimum), the mean best energy (Welch's 95% interval of the
difference contains 0) and the success probability P(E <= t) at every energy
level t the pooled sample reaches below its worst (Newcombe's interval of the
difference contains 0, Bonferroni-corrected so that the family of levels is
at 95%) must agree.  Levels are rounded to 1e-6 so that one spin
configuration counts as one level on both sides.  dSB needs no such test:
its whole trajectory is bit-exact.
"""
import numpy as np
import pytest
from scipy import stats

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_08361_amd import hsb, metrics  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    hsb.load_library()


def say(*a):
    print("[case]", *a, flush=True)


N, R, SEED, GAMMA, INTERVAL = 300, 256, 17, 0.01, 50


@pytest.mark.parametrize("kind,plan,expect", [("sk", "mixed", "fp4"), ("sk", "digits", "digits"),
                                              ("sk", "fp32", "fp32"),
                                              ("gaussian", "mixed", "digits")])
def test_bsb_long_runs_match_oracle_in_distribution(kind, plan, expect):
    if kind == "sk":
        J = synth.sk_instance(N, 23)
        c0 = np.float32(0.5 / np.sqrt(N))
        steps = 300
    else:
        J = synth.gaussian_instance(N, 24)
        c0 = np.float32(0.5)
        steps = 400
    say("bsb long-run statistics", kind, plan)
    with hsb.Context(J, precision=plan, init_amp=0.1, energy_interval=INTERVAL) as ctx:
        out = ctx.run_ex(hsb.HSB_BSB, steps, R, 1.0, float(c0), 1.0, GAMMA, SEED)
        torch.cuda.synchronize()
        assert ctx.last_plan() == expect
        eg = out["best_energy"].cpu().numpy()
    eo = oracle.run(J, oracle.BSB, 1.0, c0, 1.0, GAMMA, steps, R, seed=SEED, amp=0.1,
                    interval=INTERVAL, precision=oracle.FP64)["best_e"]
    assert np.all(np.isfinite(eg)) and np.all(np.isfinite(eo))
    lo, hi = metrics.welch_interval(eg, eo)
    say(f"mean best E: gpu {eg.mean():.4f} oracle {eo.mean():.4f}, difference in [{lo:.4f}, {hi:.4f}]")
    assert lo <= 0.0 <= hi
    pooled = np.concatenate([eg, eo])
    assert np.std(eo) > 0.0  # the comparison is not between two point masses
    levels = np.unique(np.round(pooled, 6))[:-1]
    z = stats.norm.ppf(1.0 - 0.025 / len(levels))
    for t in levels:
        tol = 1e-6 * max(1.0, abs(t))
        kg, ko = int((eg <= t + tol).sum()), int((eo <= t + tol).sum())
        plo, phi = metrics.newcombe_interval(kg, R, ko, R, z=z)
        say(f"P(E <= {t:.3f}): gpu {kg}/{R} oracle {ko}/{R}, difference in [{plo:.4f}, {phi:.4f}]")
        assert plo <= 0.0 <= phi
