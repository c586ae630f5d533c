"""The autotuner (HSB_OPT_AUTOTUNE / HSB_OPT_TILE, marked `gpu`).

Every kernel variant the tuner chooses from (operand prefetch distance of the
FP4 kernels, persistent or per-step kernel and wave height of the digit plan,
queue placement of batches) must
give bitwise the same run; the tuned choice is stored in the cache file and
reused by the next context of the same shape.  dSB runs are also the oracle's
FP32 mirror, as on every plan.
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


KEYS = ("x", "y", "spins", "energy", "best_energy", "final_energy", "best_step")

# (name, J, variant, precision, expected plan, variants, R, steps)
CASES = [
    ("dsb fp4", lambda: synth.sk_instance(700, 3), hsb.HSB_DSB, "mixed", "fp4", 3, 256, 400),
    ("bsb fp4", lambda: synth.sk_instance(700, 3), hsb.HSB_BSB, "mixed", "fp4", 2, 128, 300),
    ("bsb digits int", lambda: synth.sk_instance(600, 4) * np.float32(5), hsb.HSB_BSB, "mixed",
     "digits", 4, 96, 300),
    ("dsb digits sign", lambda: synth.sk_instance(600, 4), hsb.HSB_DSB, "digits", "digits", 4,
     96, 300),
    ("bsb digits real", lambda: synth.gaussian_instance(500, 5), hsb.HSB_BSB, "mixed", "digits",
     4, 64, 200),
]


def run(J, variant, plan, R, steps, **opts):
    N = J.shape[0]
    c0 = 0.5 / np.sqrt(N) if np.all(np.abs(J) <= 1) else 0.1 / np.sqrt(N)
    with hsb.Context(J, precision=plan, init_amp=0.1, energy_interval=50, **opts) as ctx:
        out = ctx.run_ex(variant, steps, R, 1.0, c0, 1.0, 0.02, 11, want_state=True,
                         schedule_steps=2 * steps)
        torch.cuda.synchronize()
        res = {k: v.cpu().numpy() for k, v in out.items() if hasattr(v, "cpu")}
        res["plan"] = ctx.last_plan()
        res["tile"] = int(ctx.get_option("last_tile"))
    return res, c0


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_every_variant_and_the_tuned_one_give_the_same_run(case, tmp_path, monkeypatch):
    name, mk, variant, plan, expect, nvar, R, steps = case
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("HSB_TUNE_CACHE", str(cache))
    J = mk()
    say("autotune", name)
    base, c0 = run(J, variant, plan, R, steps)
    assert base["plan"] == expect and base["tile"] == 0
    for t in range(nvar):
        got, _ = run(J, variant, plan, R, steps, tile=t)
        assert got["tile"] == t
        for k in KEYS:
            assert np.array_equal(got[k], base[k]), (name, t, k)
    with pytest.raises(hsb.HSBError) as e:
        run(J, variant, plan, R, steps, tile=nvar)
    assert e.value.code == hsb.HSB_EINVAL
    tuned, _ = run(J, variant, plan, R, steps, autotune=1)
    for k in KEYS:
        assert np.array_equal(tuned[k], base[k]), (name, "tuned", k)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1, lines
    fields = lines[0].split()
    assert int(fields[1]) == tuned["tile"] and len(fields) == 2 + nvar
    times = [float(v) for v in fields[2:]]
    assert all(t > 0 for t in times) and times[tuned["tile"]] == min(times)
    again, _ = run(J, variant, plan, R, steps, autotune=1)  # from the cache now
    assert again["tile"] == tuned["tile"] and cache.read_text().splitlines() == lines
    if variant == hsb.HSB_DSB:
        ref = oracle.run(J, oracle.DSB, 1.0, np.float32(c0), 1.0, 0.02, steps, R, seed=11,
                         amp=0.1, interval=50, precision=oracle.FP32, schedule_steps=2 * steps)
        assert np.array_equal(tuned["x"].astype(np.float64), ref["x"])
        assert np.array_equal(tuned["energy"], ref["energy"])


def test_queue_policies_and_tuned_batch_agree(tmp_path, monkeypatch):
    monkeypatch.setenv("HSB_TUNE_CACHE", str(tmp_path / "tune.txt"))
    sizes = [100, 450, 900, 1600, 2000]
    Js = [synth.sk_instance(n, 30 + k) for k, n in enumerate(sizes)]
    ctxs = [hsb.Context(J) for J in Js]
    jobs = [dict(instance=k, R=R, c0=float(np.float32(0.5 / np.sqrt(n))), gamma=0.01, seed=k + R)
            for k, n in enumerate(sizes) for R in (32, 70)]
    say("queue policies")
    res = []
    for opts in ({"tile": 0}, {"tile": 1}, {"tile": -1, "autotune": 1}):
        for k, v in opts.items():
            ctxs[0].set_option(k, v)
        outs, rc = hsb.hsb_run_batch(ctxs, jobs, hsb.HSB_DSB, 300, 1.0, 1.0, energy_interval=50)
        torch.cuda.synchronize()
        res.append([{k: v.cpu().numpy() for k, v in o.items()} for o in outs])
        if "autotune" in opts:
            assert ctxs[0].get_option("last_tile") in (0, 1)
            assert len((tmp_path / "tune.txt").read_text().splitlines()) == 1
    for other in res[1:]:
        for a, b in zip(res[0], other):
            assert np.array_equal(a["spins"], b["spins"]) and np.array_equal(a["energy"], b["energy"])
    for c in ctxs:
        c.close()
