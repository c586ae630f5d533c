#!/usr/bin/env python3
"""Benchmark: spin-updates/s of heated simulated bifurcation on one MI355X.

Workload (one bench step = one complete run of the hot path): a synthetic SK
instance N = 2000 (J_ij = +-1 equiprobable, symmetric, zero diagonal), R = 1024
replicas, Ns = 10^4 time steps of heated dSB (gamma = 0.01, dt = 1, a0 = 1,
c0 = 0.5/sqrt(N), x, y uniform in (-0.1, 0.1)), energy sampled every 100 steps,
best sample returned -- on the mixed-precision plan (FP4 field, exact).
Inputs are resident in HBM before the timed region (the J store is built once
per instance, outside it).

Reported next to it:
  - the same run on the plain FP32 plan (the baseline form) and the
    time-to-target of both plans at the same target energy;
  - the roofline of the dominant kernel (FP4 MFMA field + fused update),
    its launch duration measured with HIP events on the run's stream;
  - the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_SPINS, REPLICAS, SB_STEPS = 2000, 1024, 10000
GAMMA, DT, A0 = 0.01, 1.0, 1.0
FP4_PEAK_TFLOPS = 10100.0   # MI355X dense FP4/FP6 matrix peak
FP32_PEAK_TFLOPS = 157.3    # MI355X FP32 matrix peak


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed PMC summary, or None
    when the kernel source has changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_hbm.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        src = os.path.join(ROOT, kv["source_file"])
        with open(src, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != kv["source_sha256"]:
                return None
        return float(kv["traffic_bytes_per_dispatch"])
    except (KeyError, OSError, ValueError):
        return None


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed runs")
    ap.add_argument("--warmup", type=int, default=1, help="untimed runs")
    ap.add_argument("--sb-steps", type=int, default=SB_STEPS)
    ap.add_argument("--variant", choices=["dsb", "bsb"], default="dsb")
    ap.add_argument("--plan", choices=["mixed", "fp32", "auto"], default="mixed")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-plan comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-replicas", type=int, default=128)
    ap.add_argument("--cpu-steps", type=int, default=100)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain FP32 copy of MIB MiB (read once, written once) three "
                         "times: the reference dispatch for scaling HBM byte counters")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (replicas are "
              "independent, so several GPUs would each run a share of R)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import synth
    from paper_2203_08361_amd import hsb, metrics

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 4 * n, "kernel": "neg (FP32 elementwise)",
                          "read_bytes": 4 * n, "write_bytes": 4 * n}), flush=True)
        return 0
    N, R, Ns = N_SPINS, REPLICAS, args.sb_steps
    c0 = 0.5 / math.sqrt(N)
    variant = hsb.HSB_DSB if args.variant == "dsb" else hsb.HSB_BSB
    J = synth.sk_instance(N, 2000)
    log(f"instance N={N} built; creating context")
    ctx = hsb.Context(J, precision=args.plan, init_amp=0.1, energy_interval=100)
    plan = ctx.plan(variant)

    def one_run(seed, timing=False):
        ctx.set_option("timing", 1 if timing else 0)
        out = ctx.run_ex(variant, Ns, R, A0, c0, DT, GAMMA, seed)
        ms = ctx.get_option("kernel_ms") if timing else 0.0
        nl = int(ctx.get_option("kernel_launches")) if timing else 0
        return out, ms, nl

    for w in range(args.warmup):
        one_run(100 + w)
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    best = []
    kern_ms, kern_launches = 0.0, 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        out, ms, nl = one_run(1 + i, timing=True)
        kern_ms += ms
        kern_launches += nl
        best.append(out["best_energy"])
        log(f"timed run {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_run = 1e3 * elapsed / args.steps
    value = N * R * Ns / (elapsed / args.steps)
    best_np = torch.stack(best).cpu().numpy()

    # roofline of the dominant kernel: algorithmic work = (Ns + 1) fields of 2 N^2 R flops
    # per run (Ns steps plus the field of the final sampled state)
    flops_per_run = 2.0 * N * N * R * (Ns + 1)
    launches_per_run = kern_launches / args.steps
    avg_launch_ms = kern_ms / max(kern_launches, 1)
    achieved = flops_per_run / launches_per_run / (avg_launch_ms * 1e-3) / 1e12
    peak = FP4_PEAK_TFLOPS if plan == "mixed" else FP32_PEAK_TFLOPS
    kname = "k_dsb_fp4" if plan == "mixed" else "k_step_fp32"
    traffic = measured_traffic(kname, f"N{N}_R{R}") if Ns == SB_STEPS else None
    roofline = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 5), "traffic": traffic,
                "kernel": kname,
                "avg_launch_ms": round(avg_launch_ms, 4),
                "launches_per_run": launches_per_run}

    result = {
        "metric": "spin-updates/s (N·R·steps/s) at N=2000,R=1024; mixed-prec vs FP32 "
                  "time-to-target",
        "value": value, "unit": "spin-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_run, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "fp4xfp4->f32 field, f32 state" if plan == "mixed" else "f32",
        "data": "synthetic",
        "config": {"workload": f"SK +-1 N={N}, R={R}, {Ns} steps, heated "
                               f"{args.variant} gamma={GAMMA}, dt={DT}, {plan} plan",
                   "N": N, "R": R, "sb_steps": Ns, "variant": args.variant, "plan": plan,
                   "gamma": GAMMA, "dt": DT, "c0": c0, "energy_interval": 100},
        "roofline": roofline,
    }

    # same run on the FP32 plan and time-to-target at the pooled best energy
    if not args.no_fp32 and plan == "mixed":
        ctx.set_option("precision", "fp32")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out32, ms32, nl32 = one_run(1, timing=True)
        torch.cuda.synchronize()
        ms_run32 = 1e3 * (time.perf_counter() - t1)
        ctx.set_option("precision", args.plan)
        same = bool(torch.equal(out32["best_energy"], best[0]))
        e_star = float(best_np.min())
        tt = {}
        for name, target in (("E_best", e_star), ("E_best+0.5%", e_star + 0.005 * abs(e_star))):
            P = metrics.success_probability(best_np.ravel(), target)
            S = metrics.step_to_solution(P, Ns)
            tt[name] = {"target": target, "P": P,
                        "P_ci95": metrics.wilson_interval(int(round(P * best_np.size)),
                                                          best_np.size),
                        "step_to_solution": S,
                        "tts_s_mixed": S * ms_per_run / 1e3 / Ns,
                        "tts_s_fp32": S * ms_run32 / 1e3 / Ns}
        result["fp32_plan"] = {"value": N * R * Ns / (ms_run32 / 1e3), "ms_per_run": ms_run32,
                               "kernel_ms": ms32, "speedup_mixed": ms_run32 / ms_per_run,
                               "identical_energies": same,
                               "fp32_frac_of_peak": round(flops_per_run / (ms32 * 1e-3) / 1e12
                                                          / FP32_PEAK_TFLOPS, 4)}
        result["time_to_target"] = tt
        log(f"fp32 plan run: {ms_run32:.1f} ms")

    if not args.no_cpu_baseline:
        import oracle

        Rs, Ss = args.cpu_replicas, args.cpu_steps
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        log(f"cpu baseline: oracle FP64, {Rs} replicas x {Ss} steps on {threads} threads")
        tc = time.perf_counter()
        oracle.run(J, oracle.DSB if variant == hsb.HSB_DSB else oracle.BSB, A0, c0, DT, GAMMA,
                   Ss, Rs, seed=1, schedule_steps=Ns, precision=oracle.FP64)
        tcpu = time.perf_counter() - tc
        result["cpu_baseline"] = {"value": N * Rs * Ss / tcpu, "unit": "spin-updates/s",
                                  "cores": threads, "kind": "oracle",
                                  "sample": f"same instance, {Rs} replicas x first {Ss} of "
                                            f"{Ns} steps, FP64 oracle, {tcpu:.1f} s"}
    print(json.dumps(result), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
