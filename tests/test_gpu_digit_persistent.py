"""The digit plan's persistent kernel (marked `gpu`).

The digit plan runs the steps between two sample points in one launch
(variants 0 and 1: the two wave heights) that keeps x and y on chip, its teams
of workgroups exchanging the x digits (and, with the thermostat, the partial
sums of y^2) through L2; the per-step kernel (variants 2 and 3) computes the
same exact integer sums and the same update.  Every variant must give bitwise
the same run, for every digit combination (one- or four-digit J, x or sign
digits), with and without the thermostat, for segments of every length, for
teams that take more than one launch, and with the device-scope exchange; dSB
runs are also the oracle's FP32 mirror.
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

# (name, J, variant, precision): every combination of J digits and x digits
COMBOS = [
    ("bsb one-digit J", lambda n: synth.sk_instance(n, 41) * np.float32(5), hsb.HSB_BSB, "mixed"),
    ("dsb sign digits", lambda n: synth.sk_instance(n, 42), hsb.HSB_DSB, "digits"),
    ("bsb four-digit J", lambda n: synth.gaussian_instance(n, 43), hsb.HSB_BSB, "mixed"),
    ("dsb four-digit J", lambda n: synth.gaussian_instance(n, 44), hsb.HSB_DSB, "mixed"),
]


def c0_of(J):
    N = J.shape[0]
    return 0.5 / np.sqrt(N) if np.all(J == np.rint(J)) else 0.5


def run(J, variant, plan, steps, R, interval, tile, local=1, seed=3, **kw):
    with hsb.Context(J, precision=plan, init_amp=0.1, energy_interval=interval) as ctx:
        ctx.set_option("tile", tile)
        ctx.set_option("local_exchange", local)
        out = ctx.run_ex(variant, steps, R, 1.0, c0_of(J), 1.0, 0.02, seed, want_state=True,
                         schedule_steps=4 * steps, **kw)
        torch.cuda.synchronize()
        res = {k: v.cpu().numpy() for k, v in out.items() if hasattr(v, "cpu")}
        res["plan"] = ctx.last_plan()
        res["tile"] = int(ctx.get_option("last_tile"))
    return res


@pytest.mark.parametrize("combo", COMBOS, ids=[c[0] for c in COMBOS])
@pytest.mark.parametrize("N,R,steps,interval", [(700, 70, 130, 50), (300, 40, 37, 1)])
def test_every_variant_gives_the_same_run(combo, N, R, steps, interval):
    """interval 50: segments of 50, 50 and 30 steps; interval 1: a launch per step."""
    name, mk, variant, plan = combo
    J = mk(N)
    say("digit persistent variants", name, N, R, steps, interval)
    base = run(J, variant, plan, steps, R, interval, 0)
    assert base["plan"] == "digits" and base["tile"] == 0
    for t in (1, 2, 3):
        got = run(J, variant, plan, steps, R, interval, t)
        assert got["tile"] == t
        for k in KEYS:
            assert np.array_equal(got[k], base[k]), (name, t, k)
    if variant == hsb.HSB_DSB and name.startswith("dsb sign"):
        o = oracle.run(J, oracle.DSB, 1.0, np.float32(c0_of(J)), 1.0, 0.02, steps, R, seed=3,
                       amp=0.1, interval=interval, precision=oracle.FP32,
                       schedule_steps=4 * steps)
        assert np.array_equal(base["x"].astype(np.float64), o["x"])
        assert np.array_equal(base["energy"], o["energy"])
        assert np.array_equal(base["best_energy"], o["best_e"])


@pytest.mark.parametrize("combo", COMBOS, ids=[c[0] for c in COMBOS])
def test_thermostat_in_every_variant(combo):
    """Nose-Hoover runs (eqs. (6)-(8)): segments of 50, 50 and 30 steps; x, y
    and energies equal on every variant, and the final xi too between the
    persistent and the per-step kernel of one wave height (the same per-wave
    partials added in the same order; the two heights partition the sum
    differently: within 1e-12); dSB also equals the mirror's x and y."""
    name, mk, variant, plan = combo
    J = mk(700)
    nh = (2e-5, 0.05)  # a bath heavy enough for 700 spins (a light one lets dSB diverge)
    say("digit persistent thermostat", name)
    runs = [run(J, variant, plan, 130, 70, 50, t, nose_hoover=nh) for t in range(4)]
    base = runs[0]
    assert base["plan"] == "digits"
    for t in (1, 2, 3):
        for k in KEYS:
            assert np.array_equal(runs[t][k], base[k]), (name, t, k)
    assert np.array_equal(runs[2]["xi"], runs[0]["xi"]) and np.array_equal(runs[3]["xi"], runs[1]["xi"])
    assert np.allclose(runs[1]["xi"], runs[0]["xi"], rtol=0, atol=1e-12)
    if name.startswith("dsb sign"):
        o = oracle.run(J, oracle.DSB, 1.0, np.float32(c0_of(J)), 1.0, 0.02, 130, 70, seed=3,
                       amp=0.1, interval=50, precision=oracle.FP32, schedule_steps=520,
                       nose_hoover=nh)
        assert np.array_equal(base["x"].astype(np.float64), o["x"])
        assert np.array_equal(base["y"].astype(np.float64), o["y"])
        assert np.allclose(base["xi"], o["xi"], rtol=0, atol=1e-12)


@pytest.mark.parametrize("combo", [COMBOS[0], COMBOS[2]], ids=[COMBOS[0][0], COMBOS[2][0]])
def test_teams_beyond_one_launch_and_device_scope_exchange(combo):
    """N = 2000, R = 1100: 35 teams of 32 replicas, more than one launch holds
    (32 at either wave height), so each segment takes two launches; the
    device-scope exchange (LOCAL_EXCHANGE = 0) gives the same run."""
    name, mk, variant, plan = combo
    J = mk(2000)
    say("digit persistent two launches", name)
    base = run(J, variant, plan, 60, 1100, 25, 2)  # one launch per step
    for tile, local in ((0, 1), (0, 0)):
        got = run(J, variant, plan, 60, 1100, 25, tile, local)
        for k in KEYS:
            assert np.array_equal(got[k], base[k]), (name, tile, local, k)


@pytest.mark.parametrize("N", [4096, 8192, 8448])
def test_largest_teams_and_the_per_step_fallback(N):
    """Teams of 32 and 64 workgroups (N = 4096, 8192: two and four step flags
    per lane of the team's waves) and, beyond 8192 spins, teams too large for
    one XCD, which run one launch per step under every variant: bitwise the
    per-step kernel's run."""
    J = synth.sk_instance(N, 7)
    say("digit persistent large teams", N)
    base = run(J, hsb.HSB_DSB, "digits", 30, 64, 10, 2)
    for t in (0, 1):
        got = run(J, hsb.HSB_DSB, "digits", 30, 64, 10, t)
        assert got["plan"] == "digits"
        for k in KEYS:
            assert np.array_equal(got[k], base[k]), (N, t, k)


def test_full_size_dsb_sign_digits_against_the_mirror():
    """The bench instance on the digit plan (dSB, persistent): sampled replicas
    bitwise equal to the oracle's FP32 mirror after 300 steps of 10^4."""
    N, R = 2000, 1024
    J = synth.sk_instance(N, 2000)
    c0 = float(np.float32(0.5 / np.sqrt(N)))
    say("digit persistent full size dsb")
    with hsb.Context(J, precision="digits", energy_interval=100) as ctx:
        out = ctx.run_ex(hsb.HSB_DSB, 300, R, 1.0, c0, 1.0, 0.01, 1, want_state=True,
                         schedule_steps=10000)
        torch.cuda.synchronize()
        assert ctx.last_plan() == "digits" and ctx.get_option("last_tile") == 0
        g = {k: v.cpu().numpy() for k, v in out.items() if hasattr(v, "cpu")}
    for r in range(0, R, 97):
        o = oracle.run(J, oracle.DSB, 1.0, c0, 1.0, 0.01, 300, 1, seed=1, r0=r, amp=0.1,
                       interval=100, precision=oracle.FP32, schedule_steps=10000)
        assert np.array_equal(g["x"][r].astype(np.float64), o["x"][0]), r
        assert np.array_equal(g["y"][r].astype(np.float64), o["y"][0]), r
        assert g["best_energy"][r] == o["best_e"][0] and g["energy"][r] == o["energy"][0], r
