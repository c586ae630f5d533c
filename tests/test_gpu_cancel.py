"""Cancellation (hsb_cancel, HSB_ECANCELED, HSB_OPT_CANCELLABLE; marked `gpu`).

A cancelled run stops at a sample point, and what it returns must be exactly
what a run of that many steps returns (the same schedule): its state, its
energies, its best sample; and resuming from there must give the uncancelled
run.  A request made before the run stops it at the first sample point on
every plan (the FP4 plan's teams read the request one step before each
sample point); a request made while the run is going stops it somewhere
later, at sample points only, with each 32-replica team of the FP4 plan at
one step.
"""
import threading
import time

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_08361_amd import hsb  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    hsb.load_library()


def say(*a):
    print("[case]", *a, flush=True)


KEYS = ("x", "y", "spins", "energy", "best_energy", "final_energy", "best_step")

CASES = [(hsb.HSB_DSB, "fp32", "fp32"), (hsb.HSB_DSB, "mixed", "fp4"),
         (hsb.HSB_DSB, "digits", "digits"), (hsb.HSB_DSB, "incremental", "incremental"),
         (hsb.HSB_BSB, "fp32", "fp32"), (hsb.HSB_BSB, "mixed", "fp4"),
         (hsb.HSB_BSB, "digits", "digits")]


def host(o):
    return {k: v.cpu().numpy() for k, v in o.items() if hasattr(v, "cpu")}


@pytest.mark.parametrize("I", [100, 1])
@pytest.mark.parametrize("variant,plan,expect", CASES)
def test_request_before_the_run_stops_it_at_the_first_sample(variant, plan, expect, I):
    """I = 1 makes every step a sample point: the step that stops must not
    also record a decision for the step after it."""
    N, R, Ns = 300, 64, 1000
    J = synth.sk_instance(N, 77)
    c0 = 0.5 / np.sqrt(N)
    say("cancel before run", variant, plan, "interval", I)
    with hsb.Context(J, precision=plan, energy_interval=I, cancellable=1) as ctx:
        ctx.cancel()
        o = ctx.run_ex(variant, Ns, R, 1.0, c0, 1.0, 0.02, 5, want_state=True, allow_cancel=True)
        torch.cuda.synchronize()
        assert o["status"] == hsb.HSB_ECANCELED and ctx.last_plan() == expect
        got = host(o)
        assert np.all(got["stop_step"] == I)
        ref = host(ctx.run_ex(variant, I, R, 1.0, c0, 1.0, 0.02, 5, want_state=True,
                              schedule_steps=Ns))
        for k in KEYS:
            assert np.array_equal(got[k], ref[k]), k
        # the request is used up: the next run goes to the end
        full = ctx.run_ex(variant, Ns, R, 1.0, c0, 1.0, 0.02, 5, want_state=True,
                          allow_cancel=True)
        torch.cuda.synchronize()
        assert full["status"] == hsb.HSB_OK and bool(torch.all(full["stop_step"] == Ns))
        # resuming the cancelled run gives the uncancelled one
        res = ctx.run_ex(variant, Ns - I, R, 1.0, c0, 1.0, 0.02, 5, want_state=True,
                         x0=o["x"], y0=o["y"], start_step=I, schedule_steps=Ns)
        torch.cuda.synchronize()
        assert torch.equal(res["x"], full["x"]) and torch.equal(res["y"], full["y"])


def test_cancelled_thermostat_run_and_noalloc_run():
    N, R, Ns, I = 300, 64, 1000, 100
    J = synth.sk_instance(N, 78)
    c0 = 0.5 / np.sqrt(N)
    say("cancel thermostat / noalloc")
    with hsb.Context(J, precision="digits", energy_interval=I, cancellable=1) as ctx:
        ctx.cancel()
        o = ctx.run_ex(hsb.HSB_DSB, Ns, R, 1.0, c0, 1.0, 0.02, 5, want_state=True,
                       nose_hoover=(1e-4, 0.05), allow_cancel=True)
        ref = ctx.run_ex(hsb.HSB_DSB, I, R, 1.0, c0, 1.0, 0.02, 5, want_state=True,
                         nose_hoover=(1e-4, 0.05), schedule_steps=Ns)
        torch.cuda.synchronize()
        assert o["status"] == hsb.HSB_ECANCELED
        for k in KEYS + ("xi",):
            assert torch.equal(o[k], ref[k]), k
    with hsb.Context(J, energy_interval=I, cancellable=1) as ctx:
        ctx.cancel()
        o = ctx.run_ex(hsb.HSB_DSB, Ns, R, 1.0, c0, 1.0, 0.02, 5, want_state=True, noalloc=True,
                       allow_cancel=True)
        ref = ctx.run_ex(hsb.HSB_DSB, I, R, 1.0, c0, 1.0, 0.02, 5, want_state=True,
                         schedule_steps=Ns)
        torch.cuda.synchronize()
        assert o["status"] == hsb.HSB_ECANCELED and bool(torch.all(o["stop_step"] == I))
        for k in KEYS:
            assert torch.equal(o[k], ref[k]), k


@pytest.mark.parametrize("plan,steps,wait", [("mixed", 200000, 0.05), ("fp32", 20000, 0.3)])
def test_request_during_the_run(plan, steps, wait):
    """The run is cancelled from another thread while it goes; every replica
    stops at a sample point, and each group of replicas that stopped at step
    m equals an uncancelled run of m steps (dSB: every plan gives the exact
    trajectory, so the FP4 plan computes the reference)."""
    N, R, I = 2000, 1024, 100
    J = synth.sk_instance(N, 2000)
    c0 = 0.5 / np.sqrt(N)
    say("cancel during run", plan, steps)
    with hsb.Context(J, precision=plan, energy_interval=I, cancellable=1) as ctx:
        result = {}

        def go():
            result["o"] = ctx.run_ex(hsb.HSB_DSB, steps, R, 1.0, c0, 1.0, 0.01, 3,
                                     want_state=True, allow_cancel=True)
            torch.cuda.synchronize()

        t = threading.Thread(target=go)
        t.start()
        time.sleep(wait)
        ctx.cancel()
        t.join()
        o = host(result["o"])
    stops = o["stop_step"]
    say("  stopped at", sorted(set(stops.tolist()))[:8], "status", result["o"]["status"])
    if result["o"]["status"] == hsb.HSB_OK:
        assert np.all(stops == steps)  # finished before the request: nothing to check
        return
    assert result["o"]["status"] == hsb.HSB_ECANCELED
    assert np.all(stops % I == 0) and np.all(stops < steps) and np.all(stops > 0)
    if plan == "fp32":
        assert len(set(stops.tolist())) == 1
    for t0 in range(0, R, 32):  # one step per 32-replica team
        assert len(set(stops[t0:t0 + 32].tolist())) == 1
    with hsb.Context(J, precision="mixed", energy_interval=I) as ref_ctx:
        for m in sorted(set(stops.tolist())):
            ref = host(ref_ctx.run_ex(hsb.HSB_DSB, int(m), R, 1.0, c0, 1.0, 0.01, 3,
                                      want_state=True, schedule_steps=steps))
            sel = stops == m
            for k in KEYS:
                assert np.array_equal(o[k][sel], ref[k][sel]), (m, k)


def test_only_cancellable_contexts_take_requests():
    """HSB_OPT_CANCELLABLE = 0 (the default): hsb_cancel is refused, and runs
    of the context (which use the kernel variants without request checks)
    equal those of a cancellable context that gets no request."""
    N, R, Ns, I = 700, 64, 400, 100
    J = synth.sk_instance(N, 79)
    c0 = 0.5 / np.sqrt(N)
    say("cancel refused without the option")
    outs = []
    for opt in (0, 1):
        with hsb.Context(J, energy_interval=I, cancellable=opt) as ctx:
            assert ctx.get_option("cancellable") == opt
            if opt == 0:
                with pytest.raises(hsb.HSBError) as e:
                    ctx.cancel()
                assert e.value.code == hsb.HSB_EINVAL
            o = ctx.run_ex(hsb.HSB_DSB, Ns, R, 1.0, c0, 1.0, 0.02, 5, want_state=True)
            torch.cuda.synchronize()
            assert o["status"] == hsb.HSB_OK and ctx.last_plan() == "fp4"
            outs.append(host(o))
    for k in KEYS:
        assert np.array_equal(outs[0][k], outs[1][k]), k
