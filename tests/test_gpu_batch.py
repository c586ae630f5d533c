"""GPU parity of hsb_run_batch: many jobs over instances of uneven N.

Each job must give exactly what a separate run of its instance gives: for dSB
on +-1 couplings that is bitwise the oracle's FP32 mirror; jobs outside the
batched FP4 plan must equal hsb_run_ex on their instance.
"""
import numpy as np
import pytest

import oracle
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


def test_batch_uneven_instances_bit_exact():
    """Instances in four padded-size classes, two heating rates each, R not a
    multiple of the 32-replica team."""
    sizes = [100, 250, 300, 500, 700, 64]
    Js = [synth.sk_instance(n, 40 + k) for k, n in enumerate(sizes)]
    ctxs = [hsb.Context(J) for J in Js]
    jobs = []
    for k, n in enumerate(sizes):
        for g, R in ((0.0, 40), (0.02, 64)):
            jobs.append(dict(instance=k, R=R, c0=float(np.float32(0.5 / np.sqrt(n))), gamma=g,
                             seed=1000 + 7 * k + int(g * 100)))
    say("batch uneven", sizes)
    outs, rc = hsb.hsb_run_batch(ctxs, jobs, hsb.HSB_DSB, 300, 1.0, 1.0, init_amp=0.1,
                                 energy_interval=50)
    torch.cuda.synchronize()
    assert rc == hsb.HSB_OK
    for jd, o in zip(jobs, outs):
        J = Js[jd["instance"]]
        ref = oracle.run(J, oracle.DSB, 1.0, np.float32(jd["c0"]), 1.0, jd["gamma"], 300, jd["R"],
                         seed=jd["seed"], amp=0.1, interval=50, precision=oracle.FP32)
        assert np.array_equal(o["spins"].cpu().numpy(), ref["spins"]), jd
        assert np.array_equal(o["energy"].cpu().numpy(), ref["energy"]), jd
    for c in ctxs:
        c.close()


def test_batch_matches_single_runs_outside_fp4():
    """Jobs of a Gaussian instance (not FP4-exact: run job by job) and, for bSB,
    jobs of an FP4-exact instance (one FP4 class): the batch must return what
    hsb_run_ex returns for each job."""
    Js = [synth.sk_instance(120, 3), synth.gaussian_instance(90, 4)]
    ctxs = [hsb.Context(J) for J in Js]
    jobs = [dict(instance=0, R=24, c0=0.05, gamma=0.01, seed=5),
            dict(instance=1, R=16, c0=0.5, gamma=0.0, seed=6),
            dict(instance=0, R=8, c0=0.04, gamma=0.05, seed=7)]
    for variant in (hsb.HSB_DSB, hsb.HSB_BSB):
        say("batch vs single", variant)
        outs, rc = hsb.hsb_run_batch(ctxs, jobs, variant, 200, 1.0, 1.0, init_amp=0.1,
                                     energy_interval=40, return_best=False)
        assert rc == hsb.HSB_OK
        for jd, o in zip(jobs, outs):
            c = ctxs[jd["instance"]]
            c.set_option("init_amp", 0.1)
            c.set_option("energy_interval", 40)
            c.set_option("return_best", 0)
            ref = c.run_ex(variant, 200, jd["R"], 1.0, jd["c0"], 1.0, jd["gamma"], jd["seed"])
            torch.cuda.synchronize()
            assert torch.equal(o["spins"], ref["spins"]) and torch.equal(o["energy"],
                                                                         ref["energy"]), jd
    for c in ctxs:
        c.close()


def test_batch_rejects_invalid_jobs():
    ctx = hsb.Context(synth.sk_instance(32, 1))
    say("batch invalid")
    for bad in (dict(instance=1, R=4, c0=0.1, gamma=0.0, seed=1),
                dict(instance=0, R=0, c0=0.1, gamma=0.0, seed=1),
                dict(instance=0, R=4, c0=0.1, gamma=-1.0, seed=1)):
        with pytest.raises(hsb.HSBError) as ei:
            hsb.hsb_run_batch([ctx], [bad], hsb.HSB_DSB, 10, 1.0, 1.0)
        assert ei.value.code == hsb.HSB_EINVAL
    ctx.close()


def _scramble(outs):
    for o in outs:
        o["spins"].fill_(0)
        o["energy"].fill_(float("nan"))


def test_queue_batch_more_teams_than_the_device_holds():
    """dSB batches run as one persistent launch fed by the job queues.  48
    instances of uneven N in [100, 2000] with two jobs each of R = 64 make 192
    teams needing ~1600 workgroups, three times what the device holds at once:
    the workgroups cycle through the queues.  Every job equals the per-size
    class scheduler's result and, on a sample of jobs, the oracle's mirror."""
    sizes = [int(n) for n in synth.uneven_sizes(48, 9)]
    Js = [synth.sk_instance(n, 500 + k) for k, n in enumerate(sizes)]
    ctxs = [hsb.Context(J) for J in Js]
    jobs = [dict(instance=k, R=64, c0=float(np.float32(0.5 / np.sqrt(n))), gamma=g, seed=70 * k + q)
            for k, n in enumerate(sizes) for q, g in enumerate((0.0, 0.03))]
    say("queue batch", len(jobs), "jobs")
    res = {}
    for sched in (hsb.HSB_SCHED_QUEUE, hsb.HSB_SCHED_CLASSES):
        outs, rc = hsb.hsb_run_batch(ctxs, jobs, hsb.HSB_DSB, 200, 1.0, 1.0, init_amp=0.1,
                                     energy_interval=50, scheduler=sched)
        torch.cuda.synchronize()
        assert rc == hsb.HSB_OK
        res[sched] = [{k: v.cpu().numpy() for k, v in o.items()} for o in outs]
    for a, b in zip(res[hsb.HSB_SCHED_QUEUE], res[hsb.HSB_SCHED_CLASSES]):
        assert np.array_equal(a["spins"], b["spins"]) and np.array_equal(a["energy"], b["energy"])
    for j in (0, 17, 50, len(jobs) - 1):
        jd = jobs[j]
        J = Js[jd["instance"]]
        ref = oracle.run(J, oracle.DSB, 1.0, np.float32(jd["c0"]), 1.0, jd["gamma"], 200, 8,
                         seed=jd["seed"], amp=0.1, interval=50, precision=oracle.FP32)
        got = res[hsb.HSB_SCHED_QUEUE][j]
        assert np.array_equal(got["spins"][:8], ref["spins"]), jd
        assert np.array_equal(got["energy"][:8], ref["energy"]), jd
    for c in ctxs:
        c.close()


@pytest.mark.parametrize("steps,interval,return_best", [(0, 100, 1), (1, 1, 1), (130, 1, 0),
                                                        (257, 64, 1)])
def test_queue_batch_sampling_edges(steps, interval, return_best):
    """Zero steps (the initial state), every step sampled, final-state output
    and a last step off the sampling grid: the queue launch equals the class
    scheduler and the oracle's mirror."""
    sizes = [64, 300, 1100]
    Js = [synth.sk_instance(n, 90 + k) for k, n in enumerate(sizes)]
    ctxs = [hsb.Context(J) for J in Js]
    jobs = [dict(instance=k, R=R, c0=float(np.float32(0.5 / np.sqrt(n))), gamma=0.02, seed=3 + k)
            for k, n in enumerate(sizes) for R in (5, 33)]
    say("queue batch edges", steps, interval, return_best)
    res = {}
    for sched in (hsb.HSB_SCHED_QUEUE, hsb.HSB_SCHED_CLASSES):
        outs, rc = hsb.hsb_run_batch(ctxs, jobs, hsb.HSB_DSB, steps, 1.0, 1.0, init_amp=0.1,
                                     energy_interval=interval, return_best=bool(return_best),
                                     scheduler=sched)
        torch.cuda.synchronize()
        res[sched] = [{k: v.cpu().numpy() for k, v in o.items()} for o in outs]
    for jd, a, b in zip(jobs, res[hsb.HSB_SCHED_QUEUE], res[hsb.HSB_SCHED_CLASSES]):
        assert np.array_equal(a["spins"], b["spins"]) and np.array_equal(a["energy"], b["energy"])
        ref = oracle.run(Js[jd["instance"]], oracle.DSB, 1.0, np.float32(jd["c0"]), 1.0,
                         jd["gamma"], steps, jd["R"], seed=jd["seed"], amp=0.1, interval=interval,
                         precision=oracle.FP32, return_best=bool(return_best))
        assert np.array_equal(a["spins"], ref["spins"]) and np.array_equal(a["energy"],
                                                                           ref["energy"]), jd
    for c in ctxs:
        c.close()


def test_queue_batch_repeats_as_a_graph():
    """A batch identical to the previous one of its lead context is captured
    and replayed as one HIP graph; every replay (outputs scrambled in between,
    other work on the stream) gives the eager results.  Another batch drops it."""
    sizes = [200, 700, 1500]
    Js = [synth.sk_instance(n, 60 + k) for k, n in enumerate(sizes)]
    ctxs = [hsb.Context(J) for J in Js]
    jobs = [dict(instance=k, R=40, c0=float(np.float32(0.5 / np.sqrt(n))), gamma=0.01, seed=k)
            for k, n in enumerate(sizes)]
    say("queue batch graph")
    outs, _ = hsb.hsb_run_batch(ctxs, jobs, hsb.HSB_DSB, 300, 1.0, 1.0, energy_interval=30)
    torch.cuda.synchronize()
    eager = [{k: v.clone() for k, v in o.items()} for o in outs]
    g0 = ctxs[0].get_option("graph_launches")
    noise = torch.randn(1 << 20, device="cuda")
    for rep in range(4):
        _scramble(outs)
        noise.mul_(1.0001)  # other work queued in between
        hsb.hsb_run_batch(ctxs, jobs, hsb.HSB_DSB, 300, 1.0, 1.0, energy_interval=30, outs=outs)
        torch.cuda.synchronize()
        for a, b in zip(outs, eager):
            assert torch.equal(a["spins"], b["spins"]) and torch.equal(a["energy"], b["energy"])
    assert ctxs[0].get_option("graph_launches") - g0 == 4
    # another batch (different seed) on the same buffers: eager again, then graphed
    jobs2 = [dict(j, seed=j["seed"] + 100) for j in jobs]
    hsb.hsb_run_batch(ctxs, jobs2, hsb.HSB_DSB, 300, 1.0, 1.0, energy_interval=30, outs=outs)
    torch.cuda.synchronize()
    assert ctxs[0].get_option("graph_launches") - g0 == 4
    ref = oracle.run(Js[1], oracle.DSB, 1.0, np.float32(jobs2[1]["c0"]), 1.0, 0.01, 300, 40,
                     seed=jobs2[1]["seed"], amp=0.1, interval=30, precision=oracle.FP32)
    assert np.array_equal(outs[1]["energy"].cpu().numpy(), ref["energy"])
    for c in ctxs:
        c.close()


def test_queue_batch_reports_non_finite_and_times_its_launch():
    Js = [synth.sk_instance(40, 1), synth.sk_instance(300, 2)]
    ctxs = [hsb.Context(J) for J in Js]
    jobs = [dict(instance=0, R=8, c0=0.05, gamma=8.0, seed=1),
            dict(instance=1, R=8, c0=0.03, gamma=0.01, seed=2)]
    say("queue batch numeric")
    outs, rc = hsb.hsb_run_batch(ctxs, jobs, hsb.HSB_DSB, 400, 1.0, 1.0, allow_numeric=True)
    torch.cuda.synchronize()
    assert rc == hsb.HSB_ENUMERIC
    assert torch.all(torch.isnan(outs[0]["energy"]))
    assert not torch.any(torch.isnan(outs[1]["energy"]))
    ctxs[0].set_option("timing", 1)
    outs, rc = hsb.hsb_run_batch(ctxs, jobs[1:], hsb.HSB_DSB, 400, 1.0, 1.0)
    assert ctxs[0].get_option("kernel_launches") == 1 and ctxs[0].get_option("kernel_ms") > 0
    for c in ctxs:
        c.close()
