"""The incremental dSB field (HSB_PREC_INCREMENTAL, marked `gpu`).

For integer J the field J sgn(x) of eq. (5) is an exact integer, so carrying
it from step to step (adding 2 s_j J[:, j] for each flipped spin j) gives
bitwise the oracle's FP32 mirror, like the other plans.
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


def run(J, plan, steps, R, gamma=0.01, interval=50, seed=1, c0=None):
    N = J.shape[0]
    c0 = 0.5 / np.sqrt(N) if c0 is None else c0
    with hsb.Context(J, precision=plan, init_amp=0.1, energy_interval=interval) as ctx:
        out = ctx.run_ex(hsb.HSB_DSB, steps, R, 1.0, c0, 1.0, gamma, seed, want_state=True)
        torch.cuda.synchronize()
        res = {k: v.cpu().numpy() for k, v in out.items() if hasattr(v, "cpu")}
        res["plan"] = ctx.last_plan()
    return res


@pytest.mark.parametrize("N,R,steps,interval,scale", [(100, 16, 400, 50, 1), (130, 33, 300, 60, 1),
                                                      (300, 40, 250, 50, 5), (1, 3, 20, 7, 1),
                                                      (64, 5, 0, 10, 1)])
def test_incremental_equals_mirror(N, R, steps, interval, scale):
    J = synth.sk_instance(N, 200 + N) * np.float32(scale)
    c0 = 0.5 / np.sqrt(N) / scale
    say("incremental", N, R, steps, interval, scale)
    g = run(J, "incremental", steps, R, interval=interval, c0=c0)
    assert g["plan"] == "incremental"
    o = oracle.run(J, oracle.DSB, 1.0, np.float32(c0), 1.0, 0.01, steps, R, seed=1, amp=0.1,
                   interval=interval, precision=oracle.FP32)
    assert np.array_equal(g["x"].astype(np.float64), o["x"])
    assert np.array_equal(g["y"].astype(np.float64), o["y"])
    assert np.array_equal(g["best_energy"], o["best_e"])
    assert np.array_equal(g["final_energy"], o["final_e"])
    assert np.array_equal(g["best_step"], o["best_step"])
    assert np.array_equal(g["spins"], o["spins"])


def test_incremental_equals_the_fp4_plan():
    N, R, steps = 700, 96, 2000
    J = synth.sk_instance(N, 12)
    say("incremental vs fp4", N, R, steps)
    a = run(J, "incremental", steps, R)
    b = run(J, "mixed", steps, R)
    assert b["plan"] == "fp4"
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k


def test_incremental_unsupported_cases():
    with hsb.Context(synth.sk_instance(50, 1), precision="incremental") as ctx:
        with pytest.raises(hsb.HSBError) as e:
            ctx.run_ex(hsb.HSB_BSB, 10, 4, 1.0, 0.1, 1.0, 0.0, 1)
        assert e.value.code == hsb.HSB_EUNSUPPORTED
        with pytest.raises(hsb.HSBError) as e:
            ctx.run_ex(hsb.HSB_DSB, 10, 4, 1.0, 0.1, 1.0, 0.0, 1, nose_hoover=(1e-4, 0.1))
        assert e.value.code == hsb.HSB_EUNSUPPORTED
        assert ctx.plan(hsb.HSB_DSB) == "incremental"
    with hsb.Context(synth.gaussian_instance(50, 1), precision="incremental") as ctx:
        with pytest.raises(hsb.HSBError) as e:
            ctx.run_ex(hsb.HSB_DSB, 10, 4, 1.0, 0.5, 1.0, 0.0, 1)
        assert e.value.code == hsb.HSB_EUNSUPPORTED


def test_incremental_more_replicas_than_a_grid_dimension():
    """R = 70000 > 65535: the per-replica launches stride over the replicas
    beyond their capped grid.y; every replica equals the FP4 plan's run and a
    sample of them the oracle's FP32 mirror."""
    N, R, steps = 64, 70000, 30
    J = synth.sk_instance(N, 5)
    say("incremental R > 65535", N, R, steps)
    a = run(J, "incremental", steps, R, interval=10)
    assert a["plan"] == "incremental"
    b = run(J, "mixed", steps, R, interval=10)
    assert b["plan"] == "fp4"
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k
    for r in (0, 32767, 32768, 65535, 65536, R - 1):
        o = oracle.run(J, oracle.DSB, 1.0, np.float32(0.5 / np.sqrt(N)), 1.0, 0.01, steps, 1,
                       seed=1, amp=0.1, interval=10, precision=oracle.FP32, r0=r)
        assert np.array_equal(a["x"][r].astype(np.float64), o["x"][0]), r
        assert a["best_energy"][r] == o["best_e"][0], r
