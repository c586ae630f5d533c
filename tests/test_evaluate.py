"""Evaluation harness (paper_2203_08361_amd/evaluate.py) on the CPU.

The harness's statistics are checked on fixed trial energies against values
worked out by hand, and on trials run by the oracle on tiny instances against
brute-force ground states and the oracle's own eq. (15).
"""
import math

import numpy as np
import pytest

import oracle
import synth
from paper_2203_08361_amd import evaluate as ev
from paper_2203_08361_amd import hsb, metrics


class OracleRunner:
    """The trials of the harness run by the oracle (one oracle run per job)."""

    def __init__(self, Js, precision=oracle.FP64):
        self.Js = Js
        self.precision = precision
        self.calls = []

    def __call__(self, p, Ns, R, seeds, c0s, interval, amp):
        self.calls.append((p.name, Ns, tuple(seeds), interval))
        variant = oracle.BSB if p.variant == hsb.HSB_BSB else oracle.DSB
        return np.stack([oracle.run(J, variant, 1.0, np.float32(c0s[i]), p.dt, p.gamma, Ns, R,
                                    seed=seeds[i], amp=amp, interval=interval,
                                    precision=self.precision)["best_e"]
                         for i, J in enumerate(self.Js)])


def test_presets_are_the_papers():
    """Results, caption of the time-evolution figure."""
    got = {p.name: (p.variant, p.dt, p.c1, p.gamma) for p in ev.PRESETS}
    assert got == {"bSB": (hsb.HSB_BSB, 0.7, 0.6, 0.0), "dSB": (hsb.HSB_DSB, 1.1, 0.6, 0.0),
                   "HbSB": (hsb.HSB_BSB, 1.1, 0.9, 0.5), "HdSB": (hsb.HSB_DSB, 1.1, 0.7, 0.06)}


def test_c0_is_eq12_for_pm1_couplings():
    for N in (2, 7, 100, 700):
        J = synth.sk_instance(N, N)
        assert ev.c0_for(J, 0.6) == 0.6 / math.sqrt(N)
    # other couplings: the same field scale, c1 / (rms(J) sqrt(N))
    G = synth.gaussian_instance(300, 3)
    off = G[~np.eye(300, dtype=bool)].astype(np.float64)
    assert ev.c0_for(G, 0.5) == pytest.approx(0.5 / (np.sqrt(np.mean(off ** 2)) * np.sqrt(300)),
                                              rel=1e-15)
    assert ev.c0_for(2.0 * synth.sk_instance(50, 1), 0.5) == pytest.approx(0.5 / (2 * np.sqrt(50)))


def test_statistics_of_fixed_trials():
    """Two instances, trials given: P, S, C and medians worked out by hand."""
    # all-equal couplings: E = (N - (sum s)^2) / 2, so E in {-6, 0, 2} for
    # N = 4 (sum J = 12) and E in {-3, 1} for N = 3 (sum J = 6)
    J0 = synth.ferromagnet(4)
    J1 = synth.ferromagnet(3)
    table = {("dSB", 10): [[-6, -6, 0, 2], [-3, 1, 1, 1]],
             ("dSB", 20): [[-6, -6, -6, -6], [-3, -3, 1, 1]],
             ("HdSB", 10): [[0, 0, 0, 0], [1, 1, 1, 1]],
             ("HdSB", 20): [[-6, 0, 0, 0], [-3, -3, -3, 1]]}
    seen = []

    def runner(p, Ns, R, seeds, c0s, interval, amp):
        seen.append((p.name, Ns, tuple(seeds), interval, amp))
        return np.array(table[p.name, Ns], dtype=np.float64)

    forms = [ev.preset("dSB"), ev.preset("HdSB")]
    res = ev.evaluate([J0, J1], runner, forms, (10, 20), R=4, seed=3, interval=5)
    assert res["reference_energy"] == [-6.0, -3.0]
    assert res["reference_cut"] == [0.0, 0.0]  # all spins equal: nothing cut
    rows = {(r["form"], r["Ns"]): r for r in res["rows"]}
    d10 = rows["dSB", 10]["instances"]
    assert [q["P"] for q in d10] == [0.5, 0.25]
    assert d10[0]["S"] == pytest.approx(10 * math.log(0.01) / math.log(0.5))
    assert d10[1]["S"] == pytest.approx(10 * math.log(0.01) / math.log(0.75))
    # C = -E/2 - sum(J)/4: instance 0 trials E = -6, -6, 0, 2 -> C = 0, 0, -3, -4
    assert d10[0]["C_mean"] == -1.75 and d10[0]["C_max"] == 0.0
    assert rows["dSB", 20]["instances"][0]["S"] == 20.0  # P = 1 >= 0.99: one run
    assert math.isinf(rows["HdSB", 10]["median_S"])  # P = 0 on both
    assert rows["dSB", 10]["median_S"] == pytest.approx(
        0.5 * (d10[0]["S"] + d10[1]["S"]))
    assert res["best_Ns"] == {"dSB": {"Ns": 20, "median_S": rows["dSB", 20]["median_S"]},
                              "HdSB": {"Ns": 20, "median_S": rows["HdSB", 20]["median_S"]}}
    # the S interval is S at the ends of P's Wilson interval, in reverse order
    lo, hi = metrics.wilson_interval(2, 4)
    assert d10[0]["S_ci95"] == [metrics.step_to_solution(hi, 10), metrics.step_to_solution(lo, 10)]
    assert d10[0]["S_ci95"][0] <= d10[0]["S"] <= d10[0]["S_ci95"][1]
    # a seed per (form, N_s, instance); interval and amplitude as asked
    seeds = [s for q in seen for s in q[2]]
    assert len(set(seeds)) == len(seeds) == 8
    assert {q[3] for q in seen} == {5} and {q[4] for q in seen} == {1.0}
    # the 700-spin protocol samples the last step only
    seen.clear()
    ev.evaluate([J0, J1], runner, forms, (10, 20), R=4, final_only=True)
    assert [q[3] for q in seen] == [10, 20, 10, 20]
    # a given reference replaces the pooled best
    r2 = ev.evaluate([J0, J1], runner, forms, (10, 20), R=4, reference=[0.0, 1.0])
    assert {(r["form"], r["Ns"]): r["instances"][0]["P"] for r in r2["rows"]}[("HdSB", 10)] == 1.0


def test_real_energies_count_within_rounding():
    J = synth.gaussian_instance(20, 1)
    e = -12.345678901234
    q = ev.instance_stats([e, e * (1 + 1e-13), e * (1 - 1e-6), e + 1.0], J, e, 100)
    assert q["hits"] == 2


def test_oracle_trials_reach_brute_force_ground_states():
    """Tiny SK instances, all four forms: the pooled reference is the
    brute-force ground energy, P counts the trials that reach it, and S is the
    oracle's own eq. (15)."""
    Js = [synth.sk_instance(10, 40 + i) for i in range(3)]
    bf = [oracle.brute_force(J) for J in Js]
    ground = [b[0] for b in bf]
    run = OracleRunner(Js)
    res = ev.evaluate(Js, run, ev.PRESETS, (30, 80), R=16, seed=2, interval=10)
    assert res["reference_energy"] == pytest.approx(ground, abs=0)
    assert len(run.calls) == 8
    for row in res["rows"]:
        p = ev.preset(row["form"])
        variant = oracle.BSB if p.variant == hsb.HSB_BSB else oracle.DSB
        for i, q in enumerate(row["instances"]):
            seed = ev.trial_seed(2, ev.PRESETS.index(p), row["Ns"], i)
            E = oracle.run(Js[i], variant, 1.0, np.float32(ev.c0_for(Js[i], p.c1)), p.dt,
                           p.gamma, row["Ns"], 16, seed=seed, amp=1.0, interval=10)["best_e"]
            k = int(np.sum(E == ground[i]))
            assert q["hits"] == k
            assert q["S"] == oracle.step_to_solution(k / 16, row["Ns"])
            # eq. (14) against eq. (13) on a ground state: the maximum cut
            max_cut = oracle.cut(Js[i], bf[i][1])
            assert q["C_max"] <= max_cut and (k == 0 or q["C_max"] == max_cut)


class GroupingOracleRunner(OracleRunner):
    """The oracle runner with the grouped call (forms sharing variant and dt)."""

    def __init__(self, Js):
        super().__init__(Js)
        self.groups = []

    def run_group(self, presets, Ns, R, seeds, c0s, interval, amp):
        assert len({(p.variant, p.dt) for p in presets}) == 1
        self.groups.append(([p.name for p in presets], Ns))
        return np.stack([self(p, Ns, R, seeds[k], c0s[k], interval, amp)
                         for k, p in enumerate(presets)])


def test_grouped_forms_give_the_same_evaluation():
    """dSB and HdSB share variant and dt: a grouped runner runs them in one
    call, with the same seeds, rows and statistics as one call per form."""
    Js = [synth.sk_instance(12, 70 + i) for i in range(2)]
    plain = ev.evaluate(Js, OracleRunner(Js), ev.PRESETS, (20, 40), R=8, seed=6)
    grouped_runner = GroupingOracleRunner(Js)
    grouped = ev.evaluate(Js, grouped_runner, ev.PRESETS, (20, 40), R=8, seed=6)
    assert grouped_runner.groups == [(["dSB", "HdSB"], 20), (["dSB", "HdSB"], 40)]
    assert [(r["form"], r["Ns"]) for r in grouped["rows"]] == \
        [(p.name, ns) for p in ev.PRESETS for ns in (20, 40)]
    strip = lambda r: {k: v for k, v in r.items() if k not in ("seconds", "spin_updates_per_s")}  # noqa: E731
    assert strip(grouped) == strip(plain)


def test_sweep_ranks_by_median_S_then_by_average_cut():
    """A grid of 2 x 2 x 2 points with trial energies chosen per point: the
    ranking follows median S, and with no trial at the reference (P = 0
    everywhere) the average cut value; points sharing dt run in one call."""
    J = synth.ferromagnet(4)  # E in {-6, 0, 2}
    calls = []

    def energies(p):
        hits = {(1.0, 0.5, 0.0): 1, (1.0, 0.5, 0.1): 3, (1.0, 0.7, 0.0): 0,
                (1.0, 0.7, 0.1): 2, (1.2, 0.5, 0.0): 4, (1.2, 0.5, 0.1): 0,
                (1.2, 0.7, 0.0): 1, (1.2, 0.7, 0.1): 0}[p.dt, p.c1, p.gamma]
        zeros = {(1.0, 0.7, 0.0): 3, (1.2, 0.5, 0.1): 1}.get((p.dt, p.c1, p.gamma), 0)
        rest = 8 - hits - zeros
        return np.array([[-6.0] * hits + [0.0] * zeros + [2.0] * rest])

    class Runner:
        def __call__(self, p, Ns, R, seeds, c0s, interval, amp):
            calls.append([p.name])
            return energies(p)

        def run_group(self, presets, Ns, R, seeds, c0s, interval, amp):
            calls.append([p.name for p in presets])
            return np.stack([energies(p) for p in presets])

    res = ev.sweep([J], Runner(), hsb.HSB_DSB, 50, (1.0, 1.2), (0.5, 0.7), (0.0, 0.1), R=8)
    assert len(calls) == 2 and sorted(len(c) for c in calls) == [4, 4]
    assert res["points"] == 8 and res["criterion"] == "median S"
    assert (res["best"]["dt"], res["best"]["c1"], res["best"]["gamma"]) == (1.2, 0.5, 0.0)
    assert res["best"]["median_S"] == pytest.approx(50 * math.log(0.01) / math.log(0.5))
    order = [(q["dt"], q["c1"], q["gamma"]) for q in res["ranked"]]
    assert order[:3] == [(1.2, 0.5, 0.0), (1.0, 0.5, 0.1), (1.0, 0.7, 0.1)]
    # among the P = 0 points, the larger average cut first (more E = 0 trials)
    assert order[5:] == [(1.0, 0.7, 0.0), (1.2, 0.5, 0.1), (1.2, 0.7, 0.1)]
    # no trial at the reference: ranked by average cut alone
    low = ev.sweep([J], Runner(), hsb.HSB_DSB, 50, (1.0, 1.2), (0.5, 0.7), (0.0, 0.1), R=8,
                   reference=[-100.0])
    assert low["criterion"] == "mean C (P = 0)"
    means = [q["mean_C"] for q in low["ranked"]]
    assert means == sorted(means, reverse=True)
