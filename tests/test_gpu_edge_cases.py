"""The method's degenerate cases on every plan, against the oracle's FP32
mirror, bit for bit (marked `gpu`).

  * sgn(0) = +1, also for -0.0 (the readout and the dSB field, eq. (5)): start
    states containing +0.0 and -0.0.
  * The walls of eqs. (18)-(21) are strict: x~ landing exactly on +1 or -1
    keeps its momentum; just beyond, x is clamped and y~~ = 0, and eq. (22)
    then leaves y' = gamma dt y(t_k).  With N = 1 and J = 0 the field is 0 and
    x~ is chosen exactly (p = a0 at k = 0, a0 = dt = 1, so x~ = y in exact
    arithmetic, and every operand below is exact in FP32).
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


def gpu(J, variant, plan, steps, x0, y0, gamma, c0, interval, schedule_steps=0):
    R = x0.shape[0]
    with hsb.Context(J, precision=plan, energy_interval=interval) as ctx:
        out = ctx.run_ex(variant, steps, R, 1.0, c0, 1.0, gamma, 0, x0=torch.from_numpy(x0),
                         y0=torch.from_numpy(y0), want_state=True, schedule_steps=schedule_steps)
        torch.cuda.synchronize()
        res = {k: v.cpu().numpy() for k, v in out.items() if hasattr(v, "cpu")}
        res["plan"] = ctx.last_plan()
    return res


def mirror(J, variant, steps, x0, y0, gamma, c0, interval, schedule_steps=0):
    return oracle.run(J, variant, 1.0, np.float32(c0), 1.0, gamma, steps, x0.shape[0], x0=x0, y0=y0,
                      interval=interval, precision=oracle.FP32, schedule_steps=schedule_steps)


def same(g, o, what):
    assert np.array_equal(g["x"].astype(np.float64), o["x"]), what + " x"
    assert np.array_equal(g["y"].astype(np.float64), o["y"]), what + " y"
    assert np.array_equal(g["spins"], o["spins"]), what + " spins"
    assert np.array_equal(g["energy"], o["energy"]), what + " energy"
    assert np.array_equal(g["best_energy"], o["best_e"]), what + " best E"
    assert np.array_equal(g["final_energy"], o["final_e"]), what + " final E"
    assert np.array_equal(g["best_step"], o["best_step"]), what + " best step"


PLANS = {hsb.HSB_DSB: [("fp32", "fp32"), ("mixed", "fp4"), ("digits", "digits"),
                       ("incremental", "incremental")],
         hsb.HSB_BSB: [("fp32", "fp32"), ("mixed", "fp4"), ("digits", "digits")]}
CASES = [(v, p, e) for v in (hsb.HSB_DSB, hsb.HSB_BSB) for p, e in PLANS[v]]

# N = 1, J = 0 states: (x0, y0) and what the first step does
WALL_STATES = [
    (0.5, 1.0),     # x~ = +1 exactly: inside, y~ = 0.5 kept
    (-0.5, -1.0),   # x~ = -1 exactly
    (0.25, 1.25),   # x~ = 1.25: clamped to 1, y' = gamma dt y(t_0)
    (-0.25, -1.25),
    (0.0, 0.0),     # stays at +0
    (-0.0, 0.0),    # -0 reads as +1
    (-0.0, 0.75),
    (1.0, 0.0),     # on the wall at the start
]


@pytest.mark.parametrize("variant,plan,expect", CASES)
def test_walls_exactly_at_one_and_signed_zero(variant, plan, expect):
    J = np.zeros((1, 1), dtype=np.float32)
    x0 = np.array([[s[0]] for s in WALL_STATES], dtype=np.float32)
    y0 = np.array([[s[1]] for s in WALL_STATES], dtype=np.float32)
    assert np.signbit(x0[5, 0]) and np.signbit(x0[6, 0])
    ov = oracle.DSB if variant == hsb.HSB_DSB else oracle.BSB
    say("walls N=1", variant, plan)
    # the first step alone, then three steps sampled at every step
    for steps in (1, 3):
        g = gpu(J, variant, plan, steps, x0, y0, 0.5, 0.5, 1, schedule_steps=3)
        assert g["plan"] == expect
        o = mirror(J, ov, steps, x0, y0, 0.5, 0.5, 1, schedule_steps=3)
        same(g, o, f"{plan} steps={steps}")
    # the hand-worked first step (the walls' strict inequality)
    g = gpu(J, variant, plan, 1, x0, y0, 0.5, 0.5, 1, schedule_steps=3)
    assert g["x"][0, 0] == 1.0 and g["y"][0, 0] == 0.5 + 0.5 * 1.0
    assert g["x"][1, 0] == -1.0 and g["y"][1, 0] == -0.5 - 0.5 * 1.0
    assert g["x"][2, 0] == 1.0 and g["y"][2, 0] == 0.5 * 1.25
    assert g["x"][3, 0] == -1.0 and g["y"][3, 0] == -0.5 * 1.25
    # zero steps: the readout of the start state, sgn(-0) = +1
    g = gpu(J, variant, plan, 0, x0, y0, 0.5, 0.5, 1)
    assert g["spins"][:, 0].tolist() == [1, -1, 1, -1, 1, 1, 1, 1]


def signed_zero_state(N, R, grid):
    """Seeded x0 (amp 0.1; on a 2^-7 grid for bSB) with every fifth entry +0.0
    and every seventh -0.0; seeded y0."""
    x0, y0 = oracle.init_state(21, R, N, amp=0.1)
    if grid:
        x0 = (np.rint(x0 * 128.0) / 128.0).astype(np.float32)
    idx = np.arange(R * N).reshape(R, N)
    x0 = np.where(idx % 5 == 0, np.float32(0.0), x0)
    x0 = np.where(idx % 7 == 0, np.float32(-0.0), x0).astype(np.float32)
    assert np.signbit(x0).sum() > np.count_nonzero(x0 < 0)  # -0.0 present
    return x0, y0


@pytest.mark.parametrize("variant,plan,expect", CASES)
def test_signed_zeros_in_the_start_state(variant, plan, expect):
    N, R = 300, 40
    J = synth.sk_instance(N, 13)
    c0 = 0.5 / np.sqrt(N)
    bsb = variant == hsb.HSB_BSB
    x0, y0 = signed_zero_state(N, R, grid=bsb)
    ov = oracle.BSB if bsb else oracle.DSB
    say("signed zeros", variant, plan)
    # dSB: the field is exact on every plan, so whole runs agree; bSB: the
    # first step from a 2^-7 grid has an exact field on every plan
    for steps in ((1,) if bsb else (1, 40)):
        g = gpu(J, variant, plan, steps, x0, y0, 0.02, c0, 10, schedule_steps=1000)
        assert g["plan"] == expect
        o = mirror(J, ov, steps, x0, y0, 0.02, c0, 10, schedule_steps=1000)
        same(g, o, f"{plan} steps={steps}")
    g = gpu(J, variant, plan, 0, x0, y0, 0.02, c0, 10)
    o = mirror(J, ov, 0, x0, y0, 0.02, c0, 10)
    same(g, o, f"{plan} steps=0")
    assert np.all(g["spins"][x0 == 0.0] == 1)
