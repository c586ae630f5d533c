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
