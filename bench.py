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
  - the ballistic variant (bSB) on the same instance, mixed (integer-digit)
    plan against FP32;
  - Gaussian couplings J_ij ~ N(0, 1)/sqrt(N) at N = 2000, R = 1024, 10^4
    steps of heated bSB (c0 = 0.5): mixed (four-digit split J) plan against
    FP32, with the FP64 energies checked against the oracle's eq. (1);
  - a batched workload: 256 SK instances with N uniform in [100, 2000], each
    with 64 replicas at each of 8 heating rates (2048 jobs), 5000 steps of
    heated dSB in one hsb_run_batch call (one persistent launch), against the
    per-size class scheduler and, measured on every 8th instance, one
    FP32-plan run per instance;
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
# MI355X dense matrix-core peaks (TFLOP/s; TOP/s for int8)
KERNELS = {"fp4": ("k_dsb_fp4", 10100.0, "fp4"),
           "digits": ("k_i8_field", 5000.0, "int8"),
           "fp32": ("k_step_fp32", 157.3, "fp32")}
DTYPES = {"fp4": "fp4 x fp4 -> fp32 field, fp32 state",
          "digits": "int8 digits -> int32 field (exactly rounded), fp32 state",
          "fp32": "fp32"}


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
    ap.add_argument("--plan", choices=["mixed", "fp32", "auto", "digits"], default="mixed")
    ap.add_argument("--tile", type=int, default=-1,
                    help="kernel variant of the main runs (HSB_OPT_TILE; -1: the default)")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-plan comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bsb", action="store_true",
                    help="skip the ballistic-variant comparison of the default dSB run")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched uneven-instance workload of the default run")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched uneven-instance workload")
    ap.add_argument("--no-gaussian", action="store_true",
                    help="skip the Gaussian-coupling workload of the default run")
    ap.add_argument("--no-thermostat", action="store_true",
                    help="skip the Nose-Hoover thermostat run of the default run")
    ap.add_argument("--digits-only", action="store_true",
                    help="only the Gaussian-couplings and integer-digit legs (for profiling)")
    ap.add_argument("--thermostat-only", action="store_true",
                    help="run only the Nose-Hoover thermostat comparison")
    ap.add_argument("--no-evaluation", action="store_true",
                    help="skip the 700-spin evaluation of the four SB forms")
    ap.add_argument("--evaluation-only", action="store_true",
                    help="run only the 700-spin evaluation of the four SB forms")
    ap.add_argument("--cpu-replicas", type=int, default=128)
    ap.add_argument("--cpu-steps", type=int, default=700)
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
    if args.tile >= 0:
        ctx.set_option("tile", args.tile)

    def measure(var, steps, warmup):
        """Timed whole runs (no per-launch events), then one run with HIP-event
        timing of the dominant kernel for the roofline.  The runs write into
        the same output buffers, so that a run of the FP4 plan is launched as
        one HIP graph (captured by the library on the second identical call;
        the seed is data, not part of the graph); one untimed run before the
        warmup prepares it, as the J store is prepared before the timing."""
        dev = torch.device("cuda", 0)
        outs = {"spins": torch.empty((R, N), dtype=torch.int8, device=dev),
                "best_step": torch.empty(R, dtype=torch.int32, device=dev)}
        for k in ("energy", "best_energy", "final_energy"):
            outs[k] = torch.empty(R, dtype=torch.float64, device=dev)

        def run(seed):
            return ctx.run_ex(var, Ns, R, A0, c0, DT, GAMMA, seed, out=outs)

        ctx.set_option("timing", 0)
        run(99)
        for w in range(warmup):
            run(100 + w)
            log(f"warmup {w + 1}/{warmup} done")
        torch.cuda.synchronize()
        best = []
        g0 = ctx.get_option("graph_launches")
        t0 = time.perf_counter()
        for i in range(steps):
            best.append(run(1 + i)["best_energy"].clone())  # trials of seed 1 + i
            log(f"timed run {i + 1}/{steps} done")
        torch.cuda.synchronize()
        ms_run = 1e3 * (time.perf_counter() - t0) / steps
        graph_runs = int(ctx.get_option("graph_launches") - g0)
        plan_kind = ctx.last_plan()
        ctx.set_option("timing", 1)
        run(1)
        kern_ms = ctx.get_option("kernel_ms")
        launches = int(ctx.get_option("kernel_launches"))
        ctx.set_option("timing", 0)
        # algorithmic work of the timed kernel launches: 2 N^2 R flops per field;
        # the persistent dSB kernel also forms the field of the final sampled state
        fields = Ns + 1 if (plan_kind == "fp4" and var == hsb.HSB_DSB) else Ns
        flops = 2.0 * N * N * R * fields
        avg_ms = kern_ms / max(launches, 1)
        achieved = flops / (kern_ms * 1e-3) / 1e12
        kname, peak, peak_dtype = KERNELS[plan_kind]
        if plan_kind == "fp4" and var == hsb.HSB_BSB:
            kname = "k_bsb_fp4"
        if plan_kind == "digits" and ctx.get_option("last_tile") < 2:
            kname = "k_i8_persist"  # one launch per segment between sample points
        # per-launch HBM bytes: the persistent FP4 kernels' depend on the run
        # length; a per-step kernel's, and a digit-plan launch of one segment, do not
        wl = f"N{N}_R{R}"
        if plan_kind == "digits":  # digit-plan summaries are per variant
            wl = ("bsb_" if var == hsb.HSB_BSB else "dsb_") + wl
        traffic = (measured_traffic(kname, wl)
                   if Ns == SB_STEPS or plan_kind != "fp4" else None)
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 5), "traffic": traffic,
                "kernel": kname, "peak_dtype": peak_dtype, "avg_launch_ms": round(avg_ms, 5),
                "launches_per_run": launches}
        if var == hsb.HSB_BSB and plan_kind != "fp32":
            # matrix-core operations issued per algorithmic flop: one per x digit
            roof["issued_per_algorithmic"] = 4 if plan_kind == "digits" else 8
        return {"ms_per_run": ms_run, "value": N * R * Ns / (ms_run * 1e-3), "plan": plan_kind,
                "graph_launched_runs": graph_runs,
                "best": torch.stack(best).cpu().numpy(), "roofline": roof}

    def fp32_compare(var, mixed, n_seeds):
        """The same runs on the FP32 plan (the baseline form) and time-to-target
        on equal trials: the FP32 plan runs the first n_seeds seeds of the mixed
        plan's timed runs (seeds 1 .. n_seeds).  Where every best energy of those
        seeds is identical on both plans (dSB: the field is exact, so the
        trajectories are the same by construction) both plans have the same
        success probability, pooled over all the mixed plan's trials, and the
        time-to-target ratio is the time ratio.  Otherwise P is taken on the
        common trials of each plan, with a Wilson interval for each."""
        ctx.set_option("precision", "fp32")
        f = measure(var, n_seeds, 0)
        ctx.set_option("precision", args.plan)
        common = mixed["best"][:n_seeds]
        same = bool(np.array_equal(f["best"], common))
        e_star = float(min(mixed["best"].min(), f["best"].min()))
        pool_m = mixed["best"].ravel() if same else common.ravel()
        pool_f = pool_m if same else f["best"].ravel()
        tt = {"trials_mixed": int(pool_m.size), "trials_fp32": int(pool_f.size),
              "identical_trials": same,
              "basis": ("identical trajectories on both plans: one P, pooled over all mixed-plan "
                        "trials" if same else
                        f"P of each plan on the same {int(common.size)} trials (seeds 1..{n_seeds})")}
        for name, target in (("E_best", e_star), ("E_best+0.5%", e_star + 0.005 * abs(e_star))):
            P = metrics.success_probability(pool_m, target)
            P32 = metrics.success_probability(pool_f, target)
            S, S32 = metrics.step_to_solution(P, Ns), metrics.step_to_solution(P32, Ns)
            tts_m = S * mixed["ms_per_run"] / 1e3 / Ns
            tts_f = S32 * f["ms_per_run"] / 1e3 / Ns
            tt[name] = {"target": target, "P": P,
                        "P_ci95": metrics.wilson_interval(int(round(P * pool_m.size)), pool_m.size),
                        "P_fp32": P32,
                        "P_fp32_ci95": metrics.wilson_interval(int(round(P32 * pool_f.size)),
                                                               pool_f.size),
                        "step_to_solution": S, "step_to_solution_fp32": S32,
                        "tts_s_mixed": tts_m, "tts_s_fp32": tts_f,
                        "tts_ratio_fp32_over_mixed": (tts_f / tts_m if math.isfinite(tts_m)
                                                      and tts_m > 0 and math.isfinite(tts_f)
                                                      else None)}
        log(f"fp32 plan run: {f['ms_per_run']:.1f} ms")
        return ({"value": f["value"], "ms_per_run": f["ms_per_run"],
                 "speedup_mixed": f["ms_per_run"] / mixed["ms_per_run"],
                 "identical_energies": same, "seeds_compared": n_seeds,
                 "fp32_frac_of_peak": f["roofline"]["frac"]}, tt)

    def batch_workload():
        """2048 jobs: 256 SK instances (N uniform in [100, 2000], stream 3, seed 4),
        8 heating rates, R = 64, 5000 steps of heated dSB, c0 = 0.5/sqrt(N_i): one
        hsb_run_batch call (one persistent launch fed by the job queues; the
        repeated call is a graph launch).  Also the previous per-size class
        scheduler, and -- measured, on every 8th instance -- the baseline form:
        one FP32-plan run per instance with its 8 x 64 replicas (per-replica
        gamma), against the batch call of the same 32 instances."""
        sizes = synth.uneven_sizes(256, 4)
        gammas = [0.0, 0.0025, 0.005, 0.01, 0.02, 0.05, 0.1, 0.2]
        steps_b, R_b = 5000, 64
        log("batch: building 256 instances")
        Js = [synth.sk_instance(int(n), 10000 + k) for k, n in enumerate(sizes)]
        ctxs = [hsb.Context(Jk) for Jk in Js]

        def jobs_of(insts):
            return [dict(instance=k, R=R_b, c0=0.5 / math.sqrt(int(sizes[k])), gamma=g,
                         seed=100 * k + q) for k in insts for q, g in enumerate(gammas)]

        def work(jobs):
            su = sum(int(sizes[j["instance"]]) for j in jobs) * R_b * steps_b
            fl = sum(2.0 * int(sizes[j["instance"]]) ** 2 for j in jobs) * R_b * (steps_b + 1)
            return su, fl

        def time_batch(jobs, sched, reps):
            outs, _ = hsb.hsb_run_batch(ctxs, jobs, hsb.HSB_DSB, steps_b, A0, DT,
                                        energy_interval=100, scheduler=sched)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                hsb.hsb_run_batch(ctxs, jobs, hsb.HSB_DSB, steps_b, A0, DT, energy_interval=100,
                                  scheduler=sched, outs=outs)
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / reps

        jobs = jobs_of(range(256))
        spin_updates, flops = work(jobs)
        g0 = ctxs[0].get_option("graph_launches")
        t_batch = time_batch(jobs, hsb.HSB_SCHED_QUEUE, 3)
        graphed = int(ctxs[0].get_option("graph_launches") - g0)
        log(f"batch: {t_batch * 1e3:.1f} ms per batch (queue)")
        t_classes = time_batch(jobs, hsb.HSB_SCHED_CLASSES, 1)
        log(f"batch: {t_classes * 1e3:.1f} ms per batch (per-size classes)")
        ctxs[0].set_option("timing", 1)
        hsb.hsb_run_batch(ctxs, jobs, hsb.HSB_DSB, steps_b, A0, DT, energy_interval=100)
        kern_ms = ctxs[0].get_option("kernel_ms")
        ctxs[0].set_option("timing", 0)
        # like for like on every 8th instance: the batch call, and one FP32-plan
        # run per instance with its 8 heating rates as per-replica gamma
        sub = list(range(0, 256, 8))
        sub_jobs = jobs_of(sub)
        su_sub, _ = work(sub_jobs)
        t_sub = time_batch(sub_jobs, hsb.HSB_SCHED_QUEUE, 2)
        gam = torch.tensor(np.repeat(np.array(gammas, dtype=np.float32), R_b), device="cuda")
        t_fp32 = 0.0
        for k in sub:
            c = ctxs[k]
            c.set_option("precision", "fp32")
            c0k = 0.5 / math.sqrt(int(sizes[k]))
            c.run_ex(hsb.HSB_DSB, 100, 8 * R_b, A0, c0k, DT, 0.0, 100 * k, gamma_rep=gam)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            c.run_ex(hsb.HSB_DSB, steps_b, 8 * R_b, A0, c0k, DT, 0.0, 100 * k, gamma_rep=gam)
            torch.cuda.synchronize()
            t_fp32 += time.perf_counter() - t1
            c.set_option("precision", "auto")
        log(f"batch subset: {t_sub * 1e3:.1f} ms batched, {t_fp32 * 1e3:.1f} ms FP32 per instance")
        for c in ctxs:
            c.close()
        return {"workload": "256 SK +-1 instances, N uniform in [100, 2000] (E[N] ~ 1050), "
                            "8 gamma values {0, .0025, .005, .01, .02, .05, .1, .2} x R=64, "
                            "5000 steps heated dSB, one hsb_run_batch call",
                "jobs": len(jobs), "value": spin_updates / t_batch, "unit": "spin-updates/s",
                "ms_per_batch": t_batch * 1e3, "graph_launched_batches": graphed,
                "kernel_ms": kern_ms,
                "algorithmic_tflops": flops / t_batch / 1e12,
                "frac_fp4_peak": flops / t_batch / 1e12 / KERNELS["fp4"][1],
                "classes_scheduler_ms_per_batch": t_classes * 1e3,
                "speedup_vs_classes": t_classes / t_batch,
                "fp32_per_instance_subset": {
                    "instances": len(sub), "jobs": len(sub_jobs),
                    "batched_s": t_sub, "fp32_per_instance_s": t_fp32,
                    "speedup": t_fp32 / t_sub,
                    "basis": "measured: every 8th instance, the batch call of its 8 jobs vs one "
                             "FP32-plan hsb_run_ex per instance (R = 512, per-replica gamma)",
                    "batched_spin_updates_per_s": su_sub / t_sub,
                    "fp32_spin_updates_per_s": su_sub / t_fp32}}

    def gaussian_workload():
        """Gaussian couplings (N = 2000, seed 3), R = 1024, 10^4 steps of heated bSB,
        gamma = 0.01, c0 = 0.5 (c1 / (sigma_J sqrt(N)) with sigma_J = 1/sqrt(N))."""
        import oracle

        Jg = synth.gaussian_instance(N, 3)
        cg = hsb.Context(Jg, precision=args.plan, init_amp=0.1, energy_interval=100)
        out = {}
        for prec in (args.plan, "fp32"):
            cg.set_option("precision", prec)
            cg.run_ex(hsb.HSB_BSB, 200, R, A0, 0.5, DT, GAMMA, 100, schedule_steps=Ns)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            o = cg.run_ex(hsb.HSB_BSB, Ns, R, A0, 0.5, DT, GAMMA, 1)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0)
            out[prec] = (ms, cg.last_plan(), o)
        ms_m, plan_m, o_m = out[args.plan]
        spins = o_m["spins"].cpu().numpy()
        energy = o_m["energy"].cpu().numpy()
        rel = [abs(energy[r] - oracle.energy(Jg, spins[r])) / abs(oracle.energy(Jg, spins[r]))
               for r in range(0, R, 64)]
        cg.close()
        return {"workload": f"Gaussian J ~ N(0,1)/sqrt(N), N={N}, R={R}, {Ns} steps heated bsb "
                            f"gamma={GAMMA}, c0=0.5",
                "plan": plan_m, "value": N * R * Ns / (ms_m * 1e-3), "ms_per_run": ms_m,
                "fp32_ms_per_run": out["fp32"][0], "speedup_vs_fp32": out["fp32"][0] / ms_m,
                "fp64_energy_rel_err_max": max(rel),
                "fp64_energy_check": f"eq. (1) of the returned spins of {len(rel)} replicas "
                                     f"(every 64th) recomputed by the FP64 oracle"}

    def digits_workload():
        """The integer-digit plan (exactly rounded fields, the plan of integer J
        beyond FP4 and of real J) on the bench instance: dSB (sign digits) and
        bSB (four x digits), R = 1024, 10^4 steps, as its persistent kernel (one
        launch per segment between sample points) and as one launch per step;
        the two give the same run bit for bit."""
        cd = hsb.Context(J, precision="digits", init_amp=0.1, energy_interval=100)
        res = {}
        for vname, var in (("dsb", hsb.HSB_DSB), ("bsb", hsb.HSB_BSB)):
            row, outs = {}, {}
            for kname, tile in (("persistent", 0), ("one_launch_per_step", 2)):
                cd.set_option("tile", tile)
                cd.run_ex(var, 200, R, A0, c0, DT, GAMMA, 1, schedule_steps=Ns)  # warm-up
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                o = cd.run_ex(var, Ns, R, A0, c0, DT, GAMMA, 1, want_state=True)
                torch.cuda.synchronize()
                row[f"ms_{kname}"] = 1e3 * (time.perf_counter() - t0)
                outs[kname] = o
            a, b = outs["persistent"], outs["one_launch_per_step"]
            row["identical"] = bool(all(torch.equal(a[k], b[k])
                                        for k in ("x", "y", "spins", "best_energy", "best_step")))
            row["value"] = N * R * Ns / (row["ms_persistent"] * 1e-3)
            row["speedup_persistent"] = row["ms_one_launch_per_step"] / row["ms_persistent"]
            res[vname] = row
        cd.close()
        return {"workload": f"SK +-1 N={N}, R={R}, {Ns} steps heated dsb and bsb gamma={GAMMA}, "
                            f"integer-digit plan", "plan": "digits", **res}

    def thermostat_workload():
        """The Nose-Hoover thermostat (eqs. (6)-(8)) on the bench instance: dSB,
        R = 1024, 10^4 steps, against the heated run on the same plan: on the
        FP4 plan (the thermostat inside the persistent kernel) and on the
        integer-digit plan; and bSB on the FP4 plan."""
        # large mass (the paper's observation: xi kept negative, its rate small):
        # xi falls by at most N T / M per step, so it stays above -0.015 and
        # |xi| dt < 1 (a smaller M lets wall-pinned spins' y grow without bound)
        nh = (1e-8, 0.02)
        res = {}
        for prec, reps in ((args.plan, 3), ("digits", 1)):
            cd = hsb.Context(J, precision=prec, init_amp=0.1, energy_interval=100)
            out = {}
            for name, kw in (("heated", {}), ("nose_hoover", {"nose_hoover": nh})):
                o = cd.run_ex(hsb.HSB_DSB, Ns, R, A0, c0, DT, GAMMA, 1, **kw)
                buf = {k: v for k, v in o.items() if hasattr(v, "data_ptr")}
                cd.run_ex(hsb.HSB_DSB, Ns, R, A0, c0, DT, GAMMA, 1, out=buf, **kw)  # the graph
                torch.cuda.synchronize()
                ts = []
                for rep in range(reps):  # same buffers: repeated runs are graph launches
                    t0 = time.perf_counter()
                    o = cd.run_ex(hsb.HSB_DSB, Ns, R, A0, c0, DT, GAMMA, 2 + rep, out=buf, **kw)
                    torch.cuda.synchronize()
                    ts.append(1e3 * (time.perf_counter() - t0))
                out[name] = (float(np.mean(ts)), cd.last_plan(), o)
            xi = out["nose_hoover"][2]["xi"].cpu().numpy()
            cd.close()
            ms_h, ms_n = out["heated"][0], out["nose_hoover"][0]
            res[out["nose_hoover"][1]] = {
                "ms_per_run": ms_n, "heated_ms_per_run": ms_h, "overhead": ms_n / ms_h - 1.0,
                "runs_timed": reps, "xi_final_range": [float(xi.min()), float(xi.max())]}
        # bSB on the same instance (the thermostat inside the persistent bSB kernel)
        cb = hsb.Context(J, precision=args.plan, init_amp=0.1, energy_interval=100)
        outb = {}
        for name, kw in (("heated", {}), ("nose_hoover", {"nose_hoover": nh})):
            o = cb.run_ex(hsb.HSB_BSB, Ns, R, A0, c0, DT, GAMMA, 1, **kw)
            buf = {k: v for k, v in o.items() if hasattr(v, "data_ptr")}
            cb.run_ex(hsb.HSB_BSB, Ns, R, A0, c0, DT, GAMMA, 1, out=buf, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            o = cb.run_ex(hsb.HSB_BSB, Ns, R, A0, c0, DT, GAMMA, 2, out=buf, **kw)
            torch.cuda.synchronize()
            outb[name] = (1e3 * (time.perf_counter() - t0), cb.last_plan(), o)
        xib = outb["nose_hoover"][2]["xi"].cpu().numpy()
        cb.close()
        res["bsb_" + outb["nose_hoover"][1]] = {
            "ms_per_run": outb["nose_hoover"][0], "heated_ms_per_run": outb["heated"][0],
            "overhead": outb["nose_hoover"][0] / outb["heated"][0] - 1.0, "runs_timed": 1,
            "xi_final_range": [float(xib.min()), float(xib.max())]}
        main = res.get("fp4") or next(iter(res.values()))
        plan_main = "fp4" if "fp4" in res else next(iter(res))
        return {"workload": f"SK +-1 N={N}, R={R}, {Ns} steps dSB, Nose-Hoover 1/M={nh[0]}, "
                            f"T={nh[1]}, xi from -{GAMMA}",
                "plan": plan_main, "value": N * R * Ns / (main["ms_per_run"] * 1e-3),
                "ms_per_run": main["ms_per_run"], "heated_ms_per_run": main["heated_ms_per_run"],
                "overhead": main["overhead"], "xi_final_range": main["xi_final_range"],
                "per_plan": res}

    def incremental_late_workload():
        """The incremental dSB field (the exact int32 field, changed by the
        spins that flipped) on the last 2000 of the 10^4 steps, from the state
        the FP4 plan reached at step 8000, against the FP4 plan on the same
        steps: the results are equal bit for bit, and the time says whether
        the late schedule's few flips pay."""
        k0 = 8000
        cf = hsb.Context(J, precision=args.plan, init_amp=0.1, energy_interval=100)
        head = cf.run_ex(hsb.HSB_DSB, k0, R, A0, c0, DT, GAMMA, 1, want_state=True,
                         schedule_steps=Ns)
        x8 = head["x"].float().cpu().numpy()
        res = {}
        for name, prec in (("fp4", args.plan), ("incremental", "incremental")):
            cf.set_option("precision", prec)
            kw = dict(want_state=True, x0=head["x"], y0=head["y"], start_step=k0,
                      schedule_steps=Ns)
            cf.run_ex(hsb.HSB_DSB, Ns - k0, R, A0, c0, DT, GAMMA, 1, **kw)  # allocation, warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            o = cf.run_ex(hsb.HSB_DSB, Ns - k0, R, A0, c0, DT, GAMMA, 1, **kw)
            torch.cuda.synchronize()
            res[name] = (1e3 * (time.perf_counter() - t0), cf.last_plan(), o)
        cf.close()
        a, b = res["fp4"][2], res["incremental"][2]
        same = all(torch.equal(a[k], b[k]) for k in ("x", "y", "spins", "best_energy", "best_step"))
        flipped = float(np.mean(np.signbit(x8) != np.signbit(a["x"].cpu().numpy())))
        return {"workload": f"SK +-1 N={N}, R={R}: steps {k0}..{Ns} of a {Ns}-step heated dSB "
                            f"run, resumed from the FP4 plan's state at step {k0}",
                "ms_fp4": res["fp4"][0], "plan_fp4": res["fp4"][1],
                "ms_incremental": res["incremental"][0], "plan_incremental": res["incremental"][1],
                "identical": bool(same), "speedup_incremental": res["fp4"][0] / res["incremental"][0],
                "spins_differing_between_steps_8000_and_10000": flipped}

    def evaluation_workload():
        # the 700-spin comparison of the Results: 100 instances, the energy at
        # the last step, the four forms at the paper's parameters over a range
        # of N_s; one hsb_run_batch call per (variant, dt, N_s)
        from paper_2203_08361_amd import evaluate as ev

        n_inst, n_spins, trials, grid = 100, 700, 1024, (200, 500, 1000, 2000)
        Js = [synth.sk_instance(n_spins, 700 + i) for i in range(n_inst)]
        log(f"evaluation: {n_inst} SK instances N={n_spins}, {trials} trials, N_s {grid}")
        with ev.DeviceRunner(Js) as run:
            res = ev.evaluate(Js, run, ev.PRESETS, grid, R=trials, seed=1, final_only=True)
        best = res["best_Ns"]
        ratio = (best["HbSB"]["median_S"] / best["dSB"]["median_S"]
                 if math.isfinite(best["dSB"]["median_S"]) and best["dSB"]["median_S"] > 0
                 else None)
        return {"workload": f"{n_inst} seeded SK +-1 instances N={n_spins}, {trials} trials per "
                            f"instance, forms bSB/dSB/HbSB/HdSB at the paper's parameters, "
                            f"N_s in {list(grid)}, energy at the last step; one "
                            f"hsb_run_batch call per (variant, dt, N_s)",
                "seconds": res["seconds"], "spin_updates_per_s": res["spin_updates_per_s"],
                "reference": "per instance, the best energy any trial reached",
                "median_S": {f"{r['form']}@{r['Ns']}": r["median_S"] for r in res["rows"]},
                "mean_P": {f"{r['form']}@{r['Ns']}": r["mean_P"] for r in res["rows"]},
                "best_Ns": best, "best_median_S_HbSB_over_dSB": ratio,
                "sweep": sweep_workload(Js[:20])}

    def k2000_workload():
        # the K2000 comparison of the Results on the synthetic 2000-spin
        # instance: the four forms at the paper's parameters, N_s from 10^3 to
        # 10^4, the best of every 100 steps per trial, E* the pooled best
        from paper_2203_08361_amd import evaluate as ev

        trials, grid = 2048, (1000, 2000, 5000, 10000)
        log(f"k2000: one SK instance N={N}, {trials} trials, N_s {grid}")
        with ev.DeviceRunner([J]) as run:
            res = ev.evaluate([J], run, ev.PRESETS, grid, R=trials, seed=3, interval=100)
        rows = {f"{r['form']}@{r['Ns']}": {k: r["instances"][0][k]
                                           for k in ("P", "S", "C_mean", "C_max")}
                for r in res["rows"]}
        best = res["best_Ns"]
        d = best["dSB"]["median_S"]
        red = {f: (1.0 - best[f]["median_S"] / d) if math.isfinite(d) and d > 0 else None
               for f in ("HbSB", "HdSB")}
        return {"workload": f"SK +-1 N={N} (the bench instance), {trials} trials per form and "
                            f"N_s, N_s in {list(grid)}, best of every 100 steps",
                "seconds": res["seconds"], "spin_updates_per_s": res["spin_updates_per_s"],
                "reference_cut": res["reference_cut"][0], "per_form_and_Ns": rows,
                "best_Ns": best, "S_reduction_vs_dSB": red}

    def sweep_workload(Js):
        # the parameter search of the Results on the first 20 of those
        # instances: a 4 x 4 x 4 (dt, c1, gamma) grid per heated form, the
        # points sharing dt in one hsb_run_batch call
        from paper_2203_08361_amd import evaluate as ev

        out = {}
        with ev.DeviceRunner(Js) as run:
            for form, gammas in (("HdSB", (0.0, 0.03, 0.06, 0.12)), ("HbSB", (0.0, 0.25, 0.5, 0.75))):
                log(f"sweep: {form}, {len(Js)} instances")
                r = ev.sweep(Js, run, ev.preset(form).variant, 1000, (0.9, 1.0, 1.1, 1.25),
                             (0.5, 0.6, 0.7, 0.8), gammas, R=256, seed=2, final_only=True)
                out[form] = {"best": r["best"], "criterion": r["criterion"],
                             "seconds": r["seconds"], "spin_updates_per_s": r["spin_updates_per_s"],
                             "grid": "dt {0.9, 1.0, 1.1, 1.25} x c1 {0.5, 0.6, 0.7, 0.8} x "
                                     f"gamma {list(gammas)}, 256 trials, N_s = 1000"}
        return out

    if args.batch_only:
        print(json.dumps({"batch": batch_workload()}), flush=True)
        ctx.close()
        return 0
    if args.digits_only:
        print(json.dumps({"gaussian": gaussian_workload(), "digits": digits_workload()}),
              flush=True)
        ctx.close()
        return 0
    if args.thermostat_only:
        print(json.dumps({"thermostat": thermostat_workload()}), flush=True)
        ctx.close()
        return 0
    if args.evaluation_only:
        print(json.dumps({"evaluation": evaluation_workload(), "k2000": k2000_workload()}),
              flush=True)
        ctx.close()
        return 0

    main_res = measure(variant, args.steps, args.warmup)
    plan = main_res["plan"]
    result = {
        "metric": "spin-updates/s (N·R·steps/s) at N=2000,R=1024; mixed-prec vs FP32 "
                  "time-to-target",
        "value": main_res["value"], "unit": "spin-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_res["ms_per_run"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES[plan], "data": "synthetic",
        "config": {"workload": f"SK +-1 N={N}, R={R}, {Ns} steps, heated "
                               f"{args.variant} gamma={GAMMA}, dt={DT}, {plan} plan",
                   "N": N, "R": R, "sb_steps": Ns, "variant": args.variant, "plan": plan,
                   "gamma": GAMMA, "dt": DT, "c0": c0, "energy_interval": 100,
                   "graph_launched_runs": main_res["graph_launched_runs"]},
        "roofline": main_res["roofline"],
    }
    if not args.no_fp32 and plan != "fp32":
        result["fp32_plan"], result["time_to_target"] = fp32_compare(
            variant, main_res, 1 if variant == hsb.HSB_DSB else min(2, args.steps))
    if args.variant == "dsb" and not args.no_bsb:
        # the ballistic variant on the same instance: mixed (digit) plan vs FP32
        b = measure(hsb.HSB_BSB, 2, 1)
        bsb = {"value": b["value"], "ms_per_run": b["ms_per_run"], "plan": b["plan"],
               "dtype": DTYPES[b["plan"]], "roofline": b["roofline"]}
        if not args.no_fp32 and b["plan"] != "fp32":
            bsb["fp32_plan"], bsb["time_to_target"] = fp32_compare(hsb.HSB_BSB, b, 2)
        result["bsb"] = bsb
    if args.variant == "dsb" and not args.no_gaussian:
        result["gaussian"] = gaussian_workload()
        result["digits"] = digits_workload()
    if args.variant == "dsb" and not args.no_batch:
        result["batch"] = batch_workload()
    if args.variant == "dsb" and not args.no_thermostat:
        result["thermostat"] = thermostat_workload()
        result["incremental_late"] = incremental_late_workload()
    if args.variant == "dsb" and not args.no_evaluation:
        result["evaluation"] = evaluation_workload()
        result["k2000"] = k2000_workload()

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
