"""Evaluation of the four SB forms in the paper's terms (Results).

Every instance is solved in R trials for each form and each number of steps
N_s.  Per instance and (form, N_s) this gives
  - the average and maximum cut value C (eq. (14)) over the trials,
  - the success probability P: the fraction of trials reaching the reference
    energy E* (the paper counts trials that reach the best known cut), with
    its Wilson 95% interval,
  - the step-to-solution S of eq. (15), with the interval that P's interval
    implies (S decreases in P),
and over the instances the median S (the 700-spin comparison).  A form's
best N_s is the one with the smallest (median) S.

The reference E* of an instance is the caller's, or else the best energy that
any trial of the evaluation reached on it: the paper uses the best known cut
of K2000 and near-optimal simulated-annealing solutions for the 700-spin set,
neither of which is available here.

Protocols (Results):
  - K2000: the energy is sampled every 100 steps and the best sample is the
    trial's result (interval=100);
  - 700-spin set: the energy is evaluated at the last step only
    (final_only=True).

`sweep` is the parameter search of the Results: a grid of (dt, c1, gamma)
ranked by median S, or by the average cut where no trial reaches E*.

The trials run on the GPU through hsb_run_batch (one call per N_s and per
group of forms sharing variant and dt, over all instances); `time_evolution`
gives per-step T_inst (eq. (9)) and C traces of single runs, through the
traces of hsb_run_ex.  A runner is any callable with DeviceRunner's call
signature, so other executions of the same trials can be evaluated by the
same code.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from dataclasses import dataclass

import numpy as np

from . import hsb, metrics


@dataclass(frozen=True)
class Preset:
    name: str
    variant: int
    dt: float
    c1: float
    gamma: float


# Parameters of the K2000 comparison (Results, caption of the time-evolution
# figure), also used for the 700-spin set; a0 = 1 and c0 = c1/sqrt(N) (eq. (12)).
PRESETS = (
    Preset("bSB", hsb.HSB_BSB, 0.7, 0.6, 0.0),
    Preset("dSB", hsb.HSB_DSB, 1.1, 0.6, 0.0),
    Preset("HbSB", hsb.HSB_BSB, 1.1, 0.9, 0.5),
    Preset("HdSB", hsb.HSB_DSB, 1.1, 0.7, 0.06),
)
A0 = 1.0
AMP = 1.0  # x_i, y_i uniform in (-1, 1) (Results, after eq. (12))


def preset(name: str) -> Preset:
    for p in PRESETS:
        if p.name == name:
            return p
    raise KeyError(f"unknown preset {name!r}; known: {[p.name for p in PRESETS]}")


def c0_for(J, c1: float) -> float:
    """c0 = c1 / (sigma sqrt(N)) with sigma the root mean square of the
    off-diagonal couplings: eq. (12) for +-1 couplings (sigma = 1), and the
    same field scale for other couplings."""
    J = np.asarray(J, dtype=np.float64)
    N = J.shape[0]
    if N < 2:
        return float(c1)
    off = J[~np.eye(N, dtype=bool)]
    sigma = math.sqrt(float(np.mean(off * off)))
    return float(c1 / ((sigma if sigma > 0 else 1.0) * math.sqrt(N)))


def trial_seed(seed: int, form: int, Ns: int, instance: int) -> int:
    """Seed of the trials of one (form, N_s, instance): replica r of the job
    draws its start state from (this seed, r)."""
    return (seed * 1000003 + form * 7919 + Ns * 104729 + instance * 15485863) % (1 << 64)


class DeviceRunner:
    """Runs trials on the GPU: one hsb_run_batch call per (form, N_s), or per
    group of forms that share variant and dt, over all instances; one job of
    R trials per (form, instance)."""

    def __init__(self, Js, precision: str = "mixed"):
        import torch

        self._torch = torch
        self.Js = [np.ascontiguousarray(J, dtype=np.float32) for J in Js]
        self.ctxs = [hsb.Context(J, precision=precision) for J in self.Js]

    def __call__(self, p: Preset, Ns: int, R: int, seeds, c0s, interval: int,
                 amp: float = AMP) -> np.ndarray:
        return self.run_group([p], Ns, R, [seeds], [c0s], interval, amp)[0]

    def run_group(self, presets, Ns: int, R: int, seeds, c0s, interval: int,
                  amp: float = AMP) -> np.ndarray:
        """Several forms that share the variant and dt (c1 and gamma are per
        job) in one batch call: [len(presets)][instances][R] energies."""
        if len({(p.variant, p.dt) for p in presets}) != 1:
            raise ValueError("a group shares its variant and dt")
        n = len(self.ctxs)
        jobs = [{"instance": i, "R": R, "c0": c0s[k][i], "gamma": p.gamma, "seed": seeds[k][i]}
                for k, p in enumerate(presets) for i in range(n)]
        outs, _ = hsb.hsb_run_batch(self.ctxs, jobs, presets[0].variant, Ns, A0, presets[0].dt,
                                    init_amp=amp, energy_interval=interval, return_best=True)
        self._torch.cuda.synchronize()
        E = np.stack([o["energy"].cpu().numpy() for o in outs])
        return E.reshape(len(presets), n, R)

    def close(self):
        for c in self.ctxs:
            c.close()
        self.ctxs = []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def instance_stats(E, J, target: float, Ns: int) -> dict:
    """Statistics of one instance's trials (best energies E) at N_s steps."""
    E = np.asarray(E, dtype=np.float64)
    R = E.size
    tol = 1e-9 * max(1.0, abs(target))  # integer J: exact; real J: FP64 rounding
    k = int(np.count_nonzero(E <= target + tol))
    P = k / R
    lo, hi = metrics.wilson_interval(k, R)
    C = metrics.cut_from_energy(E, J)
    return {"P": P, "hits": k, "P_ci95": [lo, hi], "S": metrics.step_to_solution(P, Ns),
            "S_ci95": [metrics.step_to_solution(hi, Ns), metrics.step_to_solution(lo, Ns)],
            "C_mean": float(C.mean()), "C_max": float(C.max()), "E_min": float(E.min())}


def evaluate(Js, runner, presets=PRESETS, Ns_list=(200, 500, 1000, 2000), R: int = 1024,
             seed: int = 1, interval: int = 100, final_only: bool = False, reference=None,
             amp: float = AMP) -> dict:
    """Trials of every form in `presets` at every N_s of Ns_list on every
    instance of Js, and their statistics (see the module docstring).  A runner
    with a `run_group` method runs the forms that share variant and dt
    together (the trials, and so the results, are the same)."""
    Js = [np.asarray(J) for J in Js]
    n = len(Js)
    presets = list(presets)
    if len({p.name for p in presets}) != len(presets):
        raise ValueError("form names must differ")
    c0s = [[c0_for(J, p.c1) for J in Js] for p in presets]
    groups = {}
    for fi, p in enumerate(presets):
        key = (p.variant, p.dt) if hasattr(runner, "run_group") else fi
        groups.setdefault(key, []).append(fi)
    energies = {}
    t0 = time.perf_counter()
    for members in groups.values():
        for Ns in Ns_list:
            seeds = [[trial_seed(seed, fi, Ns, i) for i in range(n)] for fi in members]
            iv = Ns if final_only else interval
            if len(members) > 1:
                E = np.asarray(runner.run_group([presets[fi] for fi in members], Ns, R, seeds,
                                                [c0s[fi] for fi in members], iv, amp),
                               dtype=np.float64)
            else:
                fi = members[0]
                E = np.asarray(runner(presets[fi], Ns, R, seeds[0], c0s[fi], iv, amp),
                               dtype=np.float64)[None]
            if E.shape != (len(members), n, R):
                raise ValueError(f"runner returned shape {E.shape[1:]}, expected {(n, R)}")
            for k, fi in enumerate(members):
                energies[presets[fi].name, Ns] = E[k]
    seconds = time.perf_counter() - t0
    # rows in the order of the forms, then of N_s
    energies = {(p.name, Ns): energies[p.name, Ns] for p in presets for Ns in Ns_list}
    if reference is None:
        ref = np.min(np.stack([E.min(axis=1) for E in energies.values()]), axis=0)
    else:
        ref = np.asarray(reference, dtype=np.float64).reshape(n)
    rows = []
    for (name, Ns), E in energies.items():
        per = [instance_stats(E[i], Js[i], ref[i], Ns) for i in range(n)]
        S = np.array([q["S"] for q in per])
        rows.append({"form": name, "Ns": Ns, "median_S": float(np.median(S)),
                     "mean_P": float(np.mean([q["P"] for q in per])),
                     "mean_C": float(np.mean([q["C_mean"] for q in per])),
                     "instances": per})
    best = {}
    for p in presets:
        mine = [r for r in rows if r["form"] == p.name]
        b = min(mine, key=lambda r: (r["median_S"], r["Ns"]))
        best[p.name] = {"Ns": b["Ns"], "median_S": b["median_S"]}
    updates = sum(float(J.shape[0]) * R * Ns for J in Js for (_, Ns) in energies)
    return {"reference_energy": [float(x) for x in ref],
            "reference_cut": [float(metrics.cut_from_energy(ref[i], Js[i])) for i in range(n)],
            "trials": R, "protocol": "final" if final_only else f"best of every {interval}",
            "rows": rows, "best_Ns": best, "seconds": seconds,
            "spin_updates_per_s": updates / seconds if seconds > 0 else None}


def sweep(Js, runner, variant: int, Ns: int, dts, c1s, gammas, R: int = 256, seed: int = 1,
          interval: int = 100, final_only: bool = False, reference=None,
          amp: float = AMP) -> dict:
    """Parameter search of the Results: every (dt, c1, gamma) of the grid is
    a form, evaluated at N_s steps on every instance against one common
    reference; the forms are ranked by median S (smallest first) and, where S
    is infinite for all (P = 0, as the paper found for bSB), by the average
    cut value (largest first)."""
    grid = [Preset(f"dt={dt:g},c1={c1:g},gamma={g:g}", variant, float(dt), float(c1), float(g))
            for dt in dts for c1 in c1s for g in gammas]
    res = evaluate(Js, runner, grid, (Ns,), R, seed, interval, final_only, reference, amp)
    rows = sorted(res["rows"], key=lambda r: (r["median_S"], -r["mean_C"]))
    by_name = {p.name: p for p in grid}
    ranked = [{"dt": by_name[r["form"]].dt, "c1": by_name[r["form"]].c1,
               "gamma": by_name[r["form"]].gamma, "median_S": r["median_S"],
               "mean_P": r["mean_P"], "mean_C": r["mean_C"]} for r in rows]
    criterion = "median S" if math.isfinite(ranked[0]["median_S"]) else "mean C (P = 0)"
    return {"best": ranked[0], "criterion": criterion, "ranked": ranked, "Ns": Ns,
            "points": len(grid), "seconds": res["seconds"],
            "spin_updates_per_s": res["spin_updates_per_s"],
            "reference_energy": res["reference_energy"]}


def time_evolution(J, p: Preset, Ns: int, R: int = 1, seed: int = 1, amp: float = AMP,
                   precision: str = "mixed") -> dict:
    """Per-step instantaneous temperature (eq. (9)) and cut value (eq. (14))
    of R runs of form p: arrays [Ns + 1][R] for the states after 0 .. Ns
    steps (the time-evolution figure of the Results)."""
    import torch

    J = np.asarray(J, dtype=np.float32)
    c0 = c0_for(J, p.c1)
    with hsb.Context(J, precision=precision, init_amp=amp, energy_interval=1) as ctx:
        first = ctx.run_ex(p.variant, 0, R, A0, c0, p.dt, p.gamma, seed, traces=True,
                           schedule_steps=Ns)
        rest = ctx.run_ex(p.variant, Ns, R, A0, c0, p.dt, p.gamma, seed, traces=True)
        torch.cuda.synchronize()
        E = np.concatenate([first["trace_energy"].cpu().numpy(),
                            rest["trace_energy"].cpu().numpy()])
        T = np.concatenate([first["trace_tinst"].cpu().numpy(),
                            rest["trace_tinst"].cpu().numpy()])
    return {"T_inst": T, "C": metrics.cut_from_energy(E, J), "energy": E}


def _parse(argv):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--set", choices=("sk700", "k2000"), default="sk700",
                    help="sk700: seeded +-1 SK instances, energy at the last step; "
                         "k2000: one seeded 2000-spin SK instance, best of every 100 steps")
    ap.add_argument("--instances", type=int, default=100)
    ap.add_argument("--N", type=int, default=None)
    ap.add_argument("--trials", type=int, default=1024)
    ap.add_argument("--Ns", default="200,500,1000,2000")
    ap.add_argument("--forms", default=",".join(p.name for p in PRESETS))
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--instance-seed", type=int, default=700)
    ap.add_argument("--sweep", default=None, metavar="FORM",
                    help="instead of the comparison: search (dt, c1, gamma) for FORM's "
                         "variant at the first N_s over --dts, --c1s, --gammas")
    ap.add_argument("--dts", default="0.9,1.0,1.1,1.25")
    ap.add_argument("--c1s", default="0.5,0.6,0.7,0.8")
    ap.add_argument("--gammas", default="0,0.03,0.06,0.12")
    ap.add_argument("--out", default=None, help="write the full result as JSON here")
    return ap.parse_args(argv)


def main(argv=None) -> int:
    import synth

    a = _parse(argv)
    forms = [preset(s) for s in a.forms.split(",")]
    Ns_list = [int(s) for s in a.Ns.split(",")]
    if a.set == "sk700":
        N = a.N or 700
        Js = [synth.sk_instance(N, a.instance_seed + i) for i in range(a.instances)]
        final_only = True
    else:
        N = a.N or 2000
        Js = [synth.sk_instance(N, 2000)]
        final_only = False
    if a.sweep:
        floats = lambda t: [float(v) for v in t.split(",")]  # noqa: E731
        with DeviceRunner(Js) as run:
            res = sweep(Js, run, preset(a.sweep).variant, Ns_list[0], floats(a.dts),
                        floats(a.c1s), floats(a.gammas), a.trials, a.seed, 100, final_only)
        if a.out:
            with open(a.out, "w") as f:
                json.dump(res, f)
        print(json.dumps({k: res[k] for k in ("best", "criterion", "Ns", "points", "seconds",
                                              "spin_updates_per_s")}))
        return 0
    with DeviceRunner(Js) as run:
        res = evaluate(Js, run, forms, Ns_list, a.trials, a.seed, 100, final_only)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f)
    summary = {"set": a.set, "N": N, "instances": len(Js), "trials": a.trials,
               "seconds": round(res["seconds"], 3), "spin_updates_per_s": res["spin_updates_per_s"],
               "best_Ns": res["best_Ns"],
               "median_S": {f"{r['form']}@{r['Ns']}": r["median_S"] for r in res["rows"]}}
    print(json.dumps(summary))
    return 0


if __name__ == "__main__":
    sys.exit(main())
