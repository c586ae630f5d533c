"""Evaluation harness on the GPU (marked `gpu`): the same evaluation with its
trials run by hsb_run_batch and by the oracle.

  - dSB and HdSB: the trajectories are bitwise the oracle's FP32 mirror, so
    the whole evaluation (reference energies, every P, S, C, median) is equal.
  - bSB and HbSB: per instance and N_s, Welch's 95% interval of the difference
    of the mean best energies (GPU minus FP64 oracle) contains 0.
  - time_evolution: T_inst and C at every step equal the oracle's traces
    (dSB exactly, T_inst to FP64 summation order).
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_08361_amd import evaluate as ev  # noqa: E402
from paper_2203_08361_amd import hsb, metrics  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    hsb.load_library()


def say(*a):
    print("[case]", *a, flush=True)


class OracleRunner:
    def __init__(self, Js, precision):
        self.Js = Js
        self.precision = precision

    def __call__(self, p, Ns, R, seeds, c0s, interval, amp):
        variant = oracle.BSB if p.variant == hsb.HSB_BSB else oracle.DSB
        return np.stack([oracle.run(J, variant, 1.0, np.float32(c0s[i]), p.dt, p.gamma, Ns, R,
                                    seed=seeds[i], amp=amp, interval=interval,
                                    precision=self.precision)["best_e"]
                         for i, J in enumerate(self.Js)])


def strip(res):
    return {k: v for k, v in res.items() if k not in ("seconds", "spin_updates_per_s")}


@pytest.mark.parametrize("final_only", [False, True])
def test_dsb_forms_equal_the_oracle_evaluation(final_only):
    Js = [synth.sk_instance(N, 50 + N) for N in (64, 100, 150, 257)]
    forms = [ev.preset("dSB"), ev.preset("HdSB")]
    say("evaluation dSB forms", final_only)
    with ev.DeviceRunner(Js) as run:
        g = ev.evaluate(Js, run, forms, (60, 150), R=24, seed=4, interval=50,
                        final_only=final_only)
    o = ev.evaluate(Js, OracleRunner(Js, oracle.FP32), forms, (60, 150), R=24, seed=4,
                    interval=50, final_only=final_only)
    assert strip(g) == strip(o)
    assert g["spin_updates_per_s"] > 0


def test_bsb_forms_agree_with_the_fp64_oracle_in_distribution():
    Js = [synth.sk_instance(N, 60 + N) for N in (100, 200)]
    forms = [ev.preset("bSB"), ev.preset("HbSB")]
    R, Ns = 128, (100, 300)
    say("evaluation bSB forms")
    energies = {}

    def recording(runner, tag):
        def call(p, ns, r, seeds, c0s, interval, amp):
            E = runner(p, ns, r, seeds, c0s, interval, amp)
            energies[tag, p.name, ns] = E
            return E
        return call

    with ev.DeviceRunner(Js) as run:
        ev.evaluate(Js, recording(run, "gpu"), forms, Ns, R=R, seed=5)
    ev.evaluate(Js, recording(OracleRunner(Js, oracle.FP64), "orc"), forms, Ns, R=R, seed=5)
    for p in forms:
        for ns in Ns:
            for i in range(len(Js)):
                a, b = energies["gpu", p.name, ns][i], energies["orc", p.name, ns][i]
                lo, hi = metrics.welch_interval(a, b)
                say(f"{p.name} Ns={ns} instance {i}: mean {a.mean():.3f} vs {b.mean():.3f}, "
                    f"difference in [{lo:.3f}, {hi:.3f}]")
                assert lo <= 0.0 <= hi


@pytest.mark.parametrize("form", ["dSB", "HdSB"])
def test_time_evolution_equals_oracle_traces(form):
    N, Ns, R = 100, 200, 3
    J = synth.sk_instance(N, 77)
    p = ev.preset(form)
    say("time evolution", form)
    g = ev.time_evolution(J, p, Ns, R=R, seed=9)
    assert g["T_inst"].shape == g["C"].shape == (Ns + 1, R)
    c0 = np.float32(ev.c0_for(J, p.c1))
    o0 = oracle.run(J, oracle.DSB, 1.0, c0, p.dt, p.gamma, 0, R, seed=9, amp=1.0, interval=1,
                    precision=oracle.FP32, traces=True)
    o = oracle.run(J, oracle.DSB, 1.0, c0, p.dt, p.gamma, Ns, R, seed=9, amp=1.0, interval=1,
                   precision=oracle.FP32, traces=True)
    E = np.concatenate([o0["trace_e"], o["trace_e"]])
    T = np.concatenate([o0["trace_tinst"], o["trace_tinst"]])
    assert np.array_equal(g["energy"], E)
    assert np.array_equal(g["C"], metrics.cut_from_energy(E, J))
    np.testing.assert_allclose(g["T_inst"], T, rtol=1e-13, atol=0)


def test_time_evolution_of_the_heated_ballistic_form():
    """HbSB (gamma = 0.5) against bSB on a 2000-spin SK instance, 10^4 steps:
    the heating keeps T_inst far above bSB's at the end of the run (the
    time-evolution figure of the Results); both traces are finite."""
    N, Ns = 2000, 10000
    J = synth.sk_instance(N, 2000)
    say("time evolution HbSB vs bSB", N, Ns)
    h = ev.time_evolution(J, ev.preset("HbSB"), Ns, R=8, seed=3)
    b = ev.time_evolution(J, ev.preset("bSB"), Ns, R=8, seed=3)
    for t in (h, b):
        assert np.all(np.isfinite(t["T_inst"])) and np.all(np.isfinite(t["C"]))
    end_h = np.median(h["T_inst"][-1000:])
    end_b = np.median(b["T_inst"][-1000:])
    say(f"median T_inst over the last 1000 steps: HbSB {end_h:.3e}, bSB {end_b:.3e}")
    assert end_h > 10 * end_b


def test_dsb_sweep_equals_the_oracle_sweep():
    """(dt, c1, gamma) search for dSB: 8 points in two grouped batch calls on
    the GPU, one oracle run per point and instance; the same ranking."""
    Js = [synth.sk_instance(N, 80 + N) for N in (64, 100, 130)]
    say("dsb sweep")
    grid = ((1.0, 1.1), (0.5, 0.7), (0.0, 0.06))
    with ev.DeviceRunner(Js) as run:
        g = ev.sweep(Js, run, hsb.HSB_DSB, 80, *grid, R=16, seed=8)
    o = ev.sweep(Js, OracleRunner(Js, oracle.FP32), hsb.HSB_DSB, 80, *grid, R=16, seed=8)
    assert g["ranked"] == o["ranked"] and g["best"] == o["best"]
    assert g["reference_energy"] == o["reference_energy"]


def test_grouped_bsb_forms_equal_single_calls():
    """Forms sharing variant and dt in one batch call give exactly the trials
    of one call per form (bSB on the FP4 plan)."""
    Js = [synth.sk_instance(N, 90 + N) for N in (100, 300)]
    forms = [ev.Preset(f"g{g}", hsb.HSB_BSB, 1.1, c1, g) for c1 in (0.6, 0.9) for g in (0.0, 0.5)]
    say("grouped bsb forms")
    with ev.DeviceRunner(Js) as run:
        seeds = [[11 * k + i for i in range(2)] for k in range(4)]
        c0s = [[ev.c0_for(J, p.c1) for J in Js] for p in forms]
        grouped = run.run_group(forms, 150, 40, seeds, c0s, 50)
        single = np.stack([run(p, 150, 40, seeds[k], c0s[k], 50) for k, p in enumerate(forms)])
    assert np.array_equal(grouped, single)


def test_command_line(tmp_path, capsys):
    """python -m paper_2203_08361_amd.evaluate: the comparison and the sweep on
    a small instance set, with the full result written as JSON."""
    import json

    say("evaluate command line")
    out = tmp_path / "eval.json"
    assert ev.main(["--set", "sk700", "--instances", "3", "--N", "96", "--trials", "32",
                    "--Ns", "50,100", "--forms", "dSB,HdSB", "--out", str(out)]) == 0
    summary = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    full = json.loads(out.read_text())
    assert summary["instances"] == 3 and summary["N"] == 96
    assert set(summary["median_S"]) == {"dSB@50", "dSB@100", "HdSB@50", "HdSB@100"}
    assert len(full["rows"]) == 4 and len(full["reference_energy"]) == 3
    assert ev.main(["--set", "sk700", "--instances", "2", "--N", "64", "--trials", "16",
                    "--Ns", "60", "--sweep", "HdSB", "--dts", "1.0,1.1", "--c1s", "0.6",
                    "--gammas", "0,0.06"]) == 0
    sw = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert sw["points"] == 4 and sw["Ns"] == 60
    assert sw["best"]["dt"] in (1.0, 1.1) and sw["best"]["gamma"] in (0.0, 0.06)
