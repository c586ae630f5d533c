"""Write the stored oracle results of the full-size long runs.

The GPU tests compare runs of the bench configuration (N = 2000, R = 1024,
10^4 steps) with these files.  Computing them takes tens of minutes of CPU
time, so they are stored; this script is the only thing that writes them and
it calls nothing but the CPU oracle and the seeded instance generators.

    python tests/golden/make_longrun.py [case ...]

Cases (file longrun_<case>.json):
  dsb_sk2000_mirror  SK +-1 N = 2000 (instance seed 2000), heated dSB, gamma
                     0.01, dt 1, a0 1, c0 = 0.5/sqrt(N) (rounded to float),
                     energy every 100 steps, seed 1, replicas 16 k (k < 64) of
                     1024, on the oracle's FP32 mirror.  Stored per replica:
                     SHA-256 of the final x and y as float32 bytes, best and
                     final energy, best step.  (The field of eq. (5) is an exact
                     integer, so the GPU state must hash the same.)
  bsb_sk2000_fp64    the same instance, heated bSB, FP64, seed 1, replicas
                     0 .. 127: best and final energies, the step of the best
                     sample, and the energy of eq. (1) every 1000 steps
                     (statistical parity of long chaotic runs).
  bsb_gauss2000_fp64 Gaussian couplings N = 2000 (instance seed 3), heated
                     bSB with c0 = 0.5, FP64, seed 1, replicas 0 .. 127.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

N, STEPS, GAMMA, INTERVAL = 2000, 10000, 0.01, 100


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float32).tobytes()).hexdigest()


def seeded_rows(seed, reps, amp=0.1):
    xs, ys = zip(*(oracle.init_state(seed, 1, N, amp, r0=int(r)) for r in reps))
    return np.concatenate(xs), np.concatenate(ys)


def case_dsb_sk2000_mirror():
    J = synth.sk_instance(N, 2000)
    c0 = float(np.float32(0.5 / np.sqrt(N)))
    reps = [16 * k for k in range(64)]
    x0, y0 = seeded_rows(1, reps)
    o = oracle.run(J, oracle.DSB, 1.0, c0, 1.0, GAMMA, STEPS, len(reps), x0=x0, y0=y0,
                   interval=INTERVAL, precision=oracle.FP32)
    rows = [{"replica": r, "x_sha256": sha(o["x"][q]), "y_sha256": sha(o["y"][q]),
             "best_e": float(o["best_e"][q]), "final_e": float(o["final_e"][q]),
             "best_step": int(o["best_step"][q])} for q, r in enumerate(reps)]
    return {"instance": "synth.sk_instance(2000, 2000)", "variant": "dsb",
            "precision": "fp32 mirror", "a0": 1.0, "c0": c0, "dt": 1.0, "gamma": GAMMA,
            "steps": STEPS, "interval": INTERVAL, "seed": 1, "amp": 0.1, "replicas": rows}


def _bsb_stats(J, c0, desc):
    R = 128
    o = oracle.run(J, oracle.BSB, 1.0, c0, 1.0, GAMMA, STEPS, R, seed=1, interval=INTERVAL,
                   precision=oracle.FP64, traces=True)
    rows = list(range(9, STEPS // INTERVAL, 10))  # samples after 1000, 2000, ... steps
    return {"instance": desc, "variant": "bsb", "precision": "fp64", "a0": 1.0, "c0": c0,
            "dt": 1.0, "gamma": GAMMA, "steps": STEPS, "interval": INTERVAL, "seed": 1,
            "amp": 0.1, "replicas": list(range(R)),
            "best_e": [float(v) for v in o["best_e"]],
            "final_e": [float(v) for v in o["final_e"]],
            "best_step": [int(v) for v in o["best_step"]],
            "trace_steps": [(r + 1) * INTERVAL for r in rows],
            "trace_e": [[float(v) for v in o["trace_e"][r]] for r in rows]}


def case_bsb_sk2000_fp64():
    return _bsb_stats(synth.sk_instance(N, 2000), float(np.float32(0.5 / np.sqrt(N))),
                      "synth.sk_instance(2000, 2000)")


def case_bsb_gauss2000_fp64():
    return _bsb_stats(synth.gaussian_instance(N, 3), 0.5, "synth.gaussian_instance(2000, 3)")


CASES = {"dsb_sk2000_mirror": case_dsb_sk2000_mirror,
         "bsb_sk2000_fp64": case_bsb_sk2000_fp64,
         "bsb_gauss2000_fp64": case_bsb_gauss2000_fp64}


def main(names):
    with open(os.path.join(ROOT, "oracle", "hsb_oracle.c"), "rb") as f:
        src = hashlib.sha256(f.read()).hexdigest()
    for name in names or CASES:
        t0 = time.time()
        res = CASES[name]()
        res["oracle_source_sha256"] = src
        res["written_by"] = "tests/golden/make_longrun.py " + name
        res["cpu_seconds"] = round(time.time() - t0, 1)
        with open(os.path.join(HERE, f"longrun_{name}.json"), "w") as f:
            json.dump(res, f, indent=1)
        print(name, "done in", res["cpu_seconds"], "s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
