"""Full-size long runs against stored oracle results (marked `gpu`).

The bench configuration (N = 2000, R = 1024, 10^4 steps, energy every 100
steps) is too long for the oracle to rerun inside a test, so its results are
stored in tests/golden/longrun_*.json, written by tests/golden/make_longrun.py,
which calls the oracle only.

  * dSB: the field of eq. (5) is an exact integer, so every plan's final state
    must be bitwise the oracle's FP32 mirror: 64 replicas (every 16th of the
    1024) are compared by the SHA-256 of their final x and y, with their best
    and final energies and best step.  On the FP4 plan the run is made twice,
    the second time launched as a HIP graph, exactly as the bench times it.
  * bSB is chaotic over 10^4 steps, so the comparison is in distribution: the
    GPU's 1024 replicas (seed 2) against the FP64 oracle's 128 (seed 1, an
    independent sample), through the whole run -- the energy after every 1000
    steps, the step of the best sample, the best energy (see the test).
"""
import hashlib
import json
import os

import numpy as np
import pytest
from scipy import stats

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_08361_amd import hsb, metrics  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N, R, STEPS = 2000, 1024, 10000


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    hsb.load_library()


def say(*a):
    print("[case]", *a, flush=True)


def golden(name):
    with open(os.path.join(HERE, "golden", f"longrun_{name}.json")) as f:
        return json.load(f)


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float32).tobytes()).hexdigest()


@pytest.mark.parametrize("plan,expect", [("mixed", "fp4"), ("digits", "digits"), ("fp32", "fp32")])
def test_dsb_bench_run_matches_the_mirror(plan, expect):
    g = golden("dsb_sk2000_mirror")
    J = synth.sk_instance(N, 2000)
    say("dsb full run vs stored mirror", plan)
    dev = torch.device("cuda", 0)
    buf = {"x": torch.empty((R, N), dtype=torch.float32, device=dev),
           "y": torch.empty((R, N), dtype=torch.float32, device=dev),
           "spins": torch.empty((R, N), dtype=torch.int8, device=dev),
           "best_step": torch.empty(R, dtype=torch.int32, device=dev)}
    for k in ("energy", "best_energy", "final_energy"):
        buf[k] = torch.empty(R, dtype=torch.float64, device=dev)
    with hsb.Context(J, precision=plan, init_amp=g["amp"], energy_interval=g["interval"]) as ctx:
        outs = []
        for _ in range(2 if plan == "mixed" else 1):
            # the same output buffers: the second identical call is a graph launch
            o = ctx.run_ex(hsb.HSB_DSB, STEPS, R, g["a0"], g["c0"], g["dt"], g["gamma"], g["seed"],
                           want_state=True, out=buf)
            torch.cuda.synchronize()
            assert ctx.last_plan() == expect
            outs.append({k: v.cpu().numpy() for k, v in o.items() if hasattr(v, "cpu")})
        if plan == "mixed":
            assert ctx.get_option("graph_launches") == 1
    for out in outs:
        for row in g["replicas"]:
            r = row["replica"]
            assert sha(out["x"][r]) == row["x_sha256"], r
            assert sha(out["y"][r]) == row["y_sha256"], r
            assert out["best_energy"][r] == row["best_e"], r
            assert out["final_energy"][r] == row["final_e"], r
            assert out["best_step"][r] == row["best_step"], r
            assert out["energy"][r] == row["best_e"], r
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[-1][k]), k


def same_mean(g, o, level, what):
    """The two samples agree at `level`.  Both spread: Welch's interval of
    mean(g) - mean(o) contains 0 (widened by the rounding tolerance of an FP64
    energy sum, 1e-9 relative).  One side a single point v (up to that
    tolerance): its sample variance says nothing of the other side's tail, so
    the fractions of each side at v are compared (Newcombe's interval of their
    difference contains 0).  Both single points: the same point."""
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    tol = 1e-9 * max(1.0, abs(float(o.mean())))
    gd, od = np.ptp(g) <= tol, np.ptp(o) <= tol
    if gd and od:
        say(f"{what}: every replica at {g.mean()!r} (gpu) and {o.mean()!r} (oracle)")
        assert abs(g.mean() - o.mean()) <= tol, what
        return
    if gd or od:
        v = float((g if gd else o).mean())
        kg, ko = int((np.abs(g - v) <= tol).sum()), int((np.abs(o - v) <= tol).sum())
        vals, cnt = np.unique(np.round(g if od else o, 6), return_counts=True)
        top = sorted(zip(cnt.tolist(), vals.tolist()), reverse=True)[:4]
        lo, hi = metrics.newcombe_interval(kg, g.size, ko, o.size,
                                           z=stats.norm.ppf(0.5 + level / 2))
        say(f"{what}: at {v!r}: gpu {kg}/{g.size} oracle {ko}/{o.size}, difference in "
            f"[{lo:.4f}, {hi:.4f}]; the spread side's most frequent (count, value): {top}")
        assert lo <= 0.0 <= hi, what
        return
    lo, hi = metrics.welch_interval(g, o, level)
    say(f"{what}: gpu {g.mean():.4f} (R={g.size}) oracle {o.mean():.4f} (R={o.size}), "
        f"difference in [{lo:.4f}, {hi:.4f}]")
    assert lo - tol <= 0.0 <= hi + tol, what


@pytest.mark.parametrize("case,plan,expect", [("bsb_sk2000_fp64", "mixed", "fp4"),
                                              ("bsb_gauss2000_fp64", "mixed", "digits"),
                                              ("bsb_sk2000_fp64", "digits", "digits")])
def test_bsb_bench_runs_match_the_oracle_in_distribution(case, plan, expect):
    """Over the whole run: the energy of eq. (1) after every 1000 steps, the
    step of the best sample and the best energy agree in mean (Welch, the
    family Bonferroni-corrected to 95%), and the best energy's distribution
    agrees at the pooled deciles (Newcombe) unless every replica of both
    sides found the same energy (up to the rounding of its FP64 sum), which
    must then be equal."""
    g = golden(case)
    J = synth.sk_instance(N, 2000) if "sk" in case else synth.gaussian_instance(N, 3)
    say("bsb full run statistics", case, plan)
    with hsb.Context(J, precision=plan, init_amp=g["amp"], energy_interval=g["interval"]) as ctx:
        o = ctx.run_ex(hsb.HSB_BSB, STEPS, R, g["a0"], g["c0"], g["dt"], g["gamma"], 2,
                       traces=True)
        torch.cuda.synchronize()
        assert ctx.last_plan() == expect
        eg = o["best_energy"].cpu().numpy()
        sg = o["best_step"].cpu().numpy()
        tg = o["trace_energy"].cpu().numpy()
    eo, so = np.array(g["best_e"]), np.array(g["best_step"])
    assert np.all(np.isfinite(eg)) and np.all(np.isfinite(tg))
    rows = [m // g["interval"] - 1 for m in g["trace_steps"]]
    ntest = len(rows) + 2
    level = 1.0 - 0.05 / ntest
    for m, r, to in zip(g["trace_steps"], rows, g["trace_e"]):
        same_mean(tg[r], to, level, f"E after {m} steps")
    same_mean(sg, so, level, "step of the best sample")
    same_mean(eg, eo, level, "best energy")
    tol = 1e-9 * abs(float(eo.mean()))
    if np.ptp(eg) > tol or np.ptp(eo) > tol:
        levels = np.quantile(np.concatenate([eg, eo]), np.linspace(0.1, 0.9, 9))
        z = stats.norm.ppf(1.0 - 0.025 / len(levels))
        for t in levels:
            kg, ko = int((eg <= t).sum()), int((eo <= t).sum())
            plo, phi = metrics.newcombe_interval(kg, eg.size, ko, eo.size, z=z)
            say(f"P(E <= {t:.3f}): gpu {kg}/{eg.size} oracle {ko}/{eo.size}, "
                f"difference in [{plo:.4f}, {phi:.4f}]")
            assert plo <= 0.0 <= phi
