"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars (per the method's arithmetic):
  - dSB with integer J: the field is exact, so the single-precision trajectory
    is bitwise equal to the oracle's FP32 mirror (x, y, energies, spins), for
    the FP32 plan, the FP4 plan and the integer-digit plan.
  - bSB: per replica ||x_gpu - x_ref|| / ||x_ref|| <= 1e-5 (and for y) against
    the FP64 oracle after 1 and 50 steps.
  - energies: eq. (1) of the returned spins, exact for integer J; FP64 with
    relative error <= 1e-12 for real J.
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


def gpu_run(J, variant, plan, steps, R, seed=1, a0=1.0, c0=None, dt=1.0, gamma=0.0, amp=0.1,
            interval=100, return_best=1, **kw):
    N = J.shape[0]
    c0 = 0.5 / np.sqrt(N) if c0 is None else c0
    with hsb.Context(J, precision=plan, init_amp=amp, energy_interval=interval,
                     return_best=return_best) as ctx:
        out = ctx.run_ex(variant, steps, R, a0, c0, dt, gamma, seed, want_state=True, **kw)
        torch.cuda.synchronize()
        res = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}
        res["plan"] = ctx.plan(variant)
        res["last_plan"] = ctx.last_plan()
    return res


def oracle_run(J, variant, precision, steps, R, seed=1, a0=1.0, c0=None, dt=1.0, gamma=0.0,
               amp=0.1, interval=100, return_best=True, **kw):
    N = J.shape[0]
    c0 = 0.5 / np.sqrt(N) if c0 is None else c0
    return oracle.run(J, variant, a0, np.float32(c0), dt, gamma, steps, R, seed=seed, amp=amp,
                      interval=interval, precision=precision, return_best=return_best, **kw)


def assert_bit_exact(g, o, what=""):
    assert np.array_equal(g["x"].astype(np.float64), o["x"]), what + " x"
    assert np.array_equal(g["y"].astype(np.float64), o["y"]), what + " y"
    assert np.array_equal(g["best_energy"], o["best_e"]), what + " best E"
    assert np.array_equal(g["final_energy"], o["final_e"]), what + " final E"
    assert np.array_equal(g["best_step"], o["best_step"]), what + " best step"
    assert np.array_equal(g["spins"], o["spins"]), what + " spins"
    assert np.array_equal(g["energy"], o["energy"]), what + " energy"


# ---------------------------------------------------------------- dSB exact

@pytest.mark.parametrize("plan", ["fp32", "mixed"])
@pytest.mark.parametrize("gamma", [0.0, 0.01])
def test_dsb_small_sk_bit_exact(plan, gamma):
    """SK N=100, R=16, 2000 steps, dt=1, c0=0.5/sqrt(N), x,y in [-0.1,0.1]."""
    J = synth.sk_instance(100, 1)
    say("dsb N=100 R=16 steps=2000", plan, gamma)
    g = gpu_run(J, hsb.HSB_DSB, plan, 2000, 16, gamma=gamma)
    assert g["plan"] == ("mixed" if plan == "mixed" else "fp32")
    o = oracle_run(J, oracle.DSB, oracle.FP32, 2000, 16, gamma=gamma)
    assert_bit_exact(g, o)
    for s, e in zip(g["spins"], g["energy"]):
        assert oracle.energy(J, s) == e


@pytest.mark.parametrize("plan", ["fp32", "mixed"])
@pytest.mark.parametrize("N,R,steps,interval", [(1, 3, 40, 7), (2, 5, 30, 10), (63, 33, 300, 50),
                                                (65, 64, 250, 100), (130, 70, 120, 1),
                                                (257, 40, 90, 30)])
def test_dsb_ragged_shapes_bit_exact(plan, N, R, steps, interval):
    J = synth.sk_instance(N, N + 3)
    say("dsb ragged", plan, N, R, steps, interval)
    g = gpu_run(J, hsb.HSB_DSB, plan, steps, R, seed=N, gamma=0.02, interval=interval)
    o = oracle_run(J, oracle.DSB, oracle.FP32, steps, R, seed=N, gamma=0.02, interval=interval)
    assert_bit_exact(g, o)


@pytest.mark.parametrize("N", [700, 1100, 1500, 1800])
def test_dsb_fp4_every_padded_size_bit_exact(N):
    """Padded sizes of 12, 20, 24 and 28 K blocks of 64 spins on the FP4 plan;
    samples every 25 steps, so that runs of unsampled steps lie between them."""
    J = synth.sk_instance(N, N + 11)
    say("dsb fp4 padded size", N)
    g = gpu_run(J, hsb.HSB_DSB, "mixed", 60, 40, seed=N, gamma=0.02, interval=25)
    assert g["plan"] == "mixed"
    o = oracle_run(J, oracle.DSB, oracle.FP32, 60, 40, seed=N, gamma=0.02, interval=25)
    assert_bit_exact(g, o)


@pytest.mark.parametrize("variant", ["dsb", "bsb"])
def test_fp4_device_scope_exchange_gives_the_same_run(variant):
    """LOCAL_EXCHANGE = 0 sends every team's per-step data through device-scope
    stores and loads (with acquire/release fences for bSB), the path used when
    a team's workgroups do not share an XCD; the run must not change."""
    var = hsb.HSB_DSB if variant == "dsb" else hsb.HSB_BSB
    J = synth.sk_instance(700, 17)
    say("fp4 device-scope exchange", variant)
    outs = []
    for local in (1, 0):
        with hsb.Context(J, precision="mixed", init_amp=0.1, energy_interval=25) as ctx:
            assert ctx.get_option("local_exchange") == 1
            ctx.set_option("local_exchange", local)
            assert ctx.get_option("local_exchange") == local
            out = ctx.run_ex(var, 80, 40, 1.0, 0.5 / np.sqrt(700), 1.0, 0.02, 9, want_state=True)
            torch.cuda.synchronize()
            assert ctx.last_plan() == "fp4"
            outs.append({k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()})
            with pytest.raises(hsb.HSBError):
                ctx.set_option("local_exchange", 2)
    for k in ("x", "y", "spins", "energy", "best_energy", "final_energy", "best_step"):
        assert np.array_equal(outs[0][k], outs[1][k]), k
    if variant == "dsb":
        o = oracle_run(J, oracle.DSB, oracle.FP32, 80, 40, seed=9, gamma=0.02, interval=25)
        assert_bit_exact(outs[1], o)


@pytest.mark.parametrize("plan", ["fp32", "mixed"])
def test_dsb_zero_steps_and_final_mode(plan):
    J = synth.sk_instance(50, 2)
    say("dsb zero steps", plan)
    g = gpu_run(J, hsb.HSB_DSB, plan, 0, 8)
    o = oracle_run(J, oracle.DSB, oracle.FP32, 0, 8)
    assert_bit_exact(g, o)
    say("dsb return final", plan)
    g = gpu_run(J, hsb.HSB_DSB, plan, 333, 8, return_best=0, gamma=0.05)
    o = oracle_run(J, oracle.DSB, oracle.FP32, 333, 8, return_best=False, gamma=0.05)
    assert_bit_exact(g, o)


@pytest.mark.parametrize("plan", ["fp32", "mixed"])
def test_dsb_per_replica_gamma(plan):
    J = synth.sk_instance(120, 5)
    R = 24
    gam = np.array([0.0, 0.005, 0.01, 0.02, 0.05, 0.1, 0.2, 0.5] * 3, dtype=np.float32)
    say("dsb gamma_rep", plan)
    g = gpu_run(J, hsb.HSB_DSB, plan, 500, R, gamma_rep=torch.from_numpy(gam))
    o = oracle_run(J, oracle.DSB, oracle.FP32, 500, R, gamma=gam.astype(np.float64))
    assert_bit_exact(g, o)


@pytest.mark.parametrize("plan", ["fp32", "mixed"])
def test_dsb_resume_equals_one_run(plan):
    J = synth.sk_instance(200, 9)
    R, Ns, k = 32, 600, 250
    say("dsb resume", plan)
    full = gpu_run(J, hsb.HSB_DSB, plan, Ns, R, gamma=0.01)
    a = gpu_run(J, hsb.HSB_DSB, plan, k, R, gamma=0.01, schedule_steps=Ns)
    b = gpu_run(J, hsb.HSB_DSB, plan, Ns - k, R, gamma=0.01, start_step=k, schedule_steps=Ns,
                x0=torch.from_numpy(a["x"]), y0=torch.from_numpy(a["y"]))
    assert np.array_equal(b["x"], full["x"]) and np.array_equal(b["y"], full["y"])
    assert np.array_equal(b["final_energy"], full["final_energy"])
    o = oracle_run(J, oracle.DSB, oracle.FP32, Ns - k, R, gamma=0.01, start_step=k,
                   schedule_steps=Ns, x0=a["x"], y0=a["y"])
    assert_bit_exact(b, o)


def test_dsb_plans_agree_and_are_deterministic():
    J = synth.sk_instance(300, 4)
    say("dsb determinism")
    a = gpu_run(J, hsb.HSB_DSB, "mixed", 400, 64, gamma=0.03, seed=77)
    b = gpu_run(J, hsb.HSB_DSB, "mixed", 400, 64, gamma=0.03, seed=77)
    c = gpu_run(J, hsb.HSB_DSB, "fp32", 400, 64, gamma=0.03, seed=77)
    for k in ("x", "y", "spins", "energy", "best_step"):
        assert np.array_equal(a[k], b[k]) and np.array_equal(a[k], c[k]), k
    # replica r depends only on (seed, r): a run of fewer replicas is a prefix
    d = gpu_run(J, hsb.HSB_DSB, "mixed", 400, 37, gamma=0.03, seed=77)
    assert np.array_equal(d["x"], a["x"][:37]) and np.array_equal(d["energy"], a["energy"][:37])


def int_instance(N, seed, scale=5):
    """Integer couplings +-scale: exact in int8 but not in FP4 (scale 5), so the
    mixed precision option takes the integer-digit plan."""
    return synth.sk_instance(N, seed) * np.float32(scale)


@pytest.mark.parametrize("N,R,steps,interval", [(1, 3, 40, 7), (63, 33, 300, 50),
                                                (65, 64, 250, 100), (300, 40, 400, 1),
                                                (513, 96, 200, 60)])
def test_dsb_digit_plan_bit_exact(N, R, steps, interval):
    J = int_instance(N, N + 11)
    c0 = 0.1 / np.sqrt(N)
    say("dsb digits", N, R, steps, interval)
    g = gpu_run(J, hsb.HSB_DSB, "mixed", steps, R, seed=N, c0=c0, gamma=0.02, interval=interval)
    assert g["last_plan"] == ("fp4" if N == 1 else "digits")  # N = 1: J = 0 is FP4-exact
    o = oracle_run(J, oracle.DSB, oracle.FP32, steps, R, seed=N, c0=c0, gamma=0.02,
                   interval=interval)
    assert_bit_exact(g, o)


def test_dsb_digit_plan_beyond_fp4_size():
    """N = 2100 > 2048: the FP4 plan does not apply, the digit plan is exact."""
    J = synth.sk_instance(2100, 21)
    say("dsb digits N=2100")
    g = gpu_run(J, hsb.HSB_DSB, "mixed", 150, 40, seed=5, gamma=0.01, schedule_steps=2000,
                interval=50)
    assert g["last_plan"] == "digits"
    o = oracle_run(J, oracle.DSB, oracle.FP32, 150, 40, seed=5, gamma=0.01, schedule_steps=2000,
                   interval=50)
    assert_bit_exact(g, o)


def test_dsb_digit_plan_resume_and_gamma_rep():
    J = int_instance(200, 8)
    c0 = 0.1 / np.sqrt(200)
    R, Ns, k = 32, 500, 170
    gam = np.linspace(0.0, 0.1, R).astype(np.float32)
    say("dsb digits resume")
    full = gpu_run(J, hsb.HSB_DSB, "mixed", Ns, R, c0=c0, gamma_rep=torch.from_numpy(gam))
    a = gpu_run(J, hsb.HSB_DSB, "mixed", k, R, c0=c0, schedule_steps=Ns,
                gamma_rep=torch.from_numpy(gam))
    b = gpu_run(J, hsb.HSB_DSB, "mixed", Ns - k, R, c0=c0, start_step=k, schedule_steps=Ns,
                x0=torch.from_numpy(a["x"]), y0=torch.from_numpy(a["y"]),
                gamma_rep=torch.from_numpy(gam))
    assert np.array_equal(b["x"], full["x"]) and np.array_equal(b["y"], full["y"])
    o = oracle_run(J, oracle.DSB, oracle.FP32, Ns, R, c0=c0, gamma=gam.astype(np.float64))
    assert_bit_exact(full, o)


# --------------------------------------------------- full-size (N=2000, R=1024)

@pytest.mark.parametrize("plan", ["mixed", "fp32"])
def test_dsb_full_size_sampled_replicas(plan):
    """N=2000, R=1024 over the first 300 steps of the 10^4-step schedule; the
    oracle recomputes sampled replicas one by one (replica r depends only on (seed, r))."""
    J = synth.sk_instance(2000, 2000)
    say("dsb full size", plan)
    g = gpu_run(J, hsb.HSB_DSB, plan, 300, 1024, seed=3, gamma=0.01, schedule_steps=10000)
    for r in (0, 1, 517, 1023):
        o = oracle_run(J, oracle.DSB, oracle.FP32, 300, 1, seed=3, gamma=0.01, r0=r,
                       schedule_steps=10000)
        assert np.array_equal(g["x"][r].astype(np.float64), o["x"][0]), r
        assert np.array_equal(g["y"][r].astype(np.float64), o["y"][0]), r
        assert g["best_energy"][r] == o["best_e"][0] and g["final_energy"][r] == o["final_e"][0]
    # every returned energy is eq. (1) of the returned spins (check a sample)
    for r in range(0, 1024, 97):
        assert oracle.energy(J, g["spins"][r]) == g["energy"][r]


# ---------------------------------------------------------------- bSB 1e-5

def rel_err(a, b):
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


# bSB plans: "fp32", "fp4" (mixed on +-1 couplings: FP4 J x base-8 FP4 digits of x) and
# "digits" (mixed on +-5 couplings, not FP4-exact, or forced: int8 digits)
BSB_PLANS = [("fp32", 1), ("mixed", 1), ("mixed", 5), ("digits", 1)]


def bsb_case(plan, scale, N, seed):
    J = synth.sk_instance(N, seed) * np.float32(scale)
    expect = {"fp32": "fp32", "digits": "digits"}.get(plan, "fp4" if scale == 1 else "digits")
    return J, 0.5 / np.sqrt(N) / scale, expect


@pytest.mark.parametrize("plan,scale", BSB_PLANS)
@pytest.mark.parametrize("steps", [1, 50])
@pytest.mark.parametrize("gamma", [0.0, 0.01])
def test_bsb_trajectory_within_1e5(plan, scale, steps, gamma):
    J, c0, expect = bsb_case(plan, scale, 100, 1)
    say("bsb N=100", plan, scale, steps, gamma)
    g = gpu_run(J, hsb.HSB_BSB, plan, steps, 16, c0=c0, gamma=gamma, schedule_steps=2000)
    assert g["last_plan"] == expect
    o = oracle_run(J, oracle.BSB, oracle.FP64, steps, 16, c0=c0, gamma=gamma,
                   schedule_steps=2000)
    assert rel_err(g["x"], o["x"]).max() <= 1e-5
    assert rel_err(g["y"], o["y"]).max() <= 1e-5


@pytest.mark.parametrize("plan,scale", BSB_PLANS)
def test_bsb_full_size_sampled_replicas(plan, scale):
    J, c0, expect = bsb_case(plan, scale, 2000, 2000)
    say("bsb full size", plan, scale)
    g = gpu_run(J, hsb.HSB_BSB, plan, 50, 1024, seed=3, c0=c0, gamma=0.01, schedule_steps=10000)
    assert g["last_plan"] == expect
    for r in (0, 700, 1023):
        o = oracle_run(J, oracle.BSB, oracle.FP64, 50, 1, seed=3, c0=c0, gamma=0.01, r0=r,
                       schedule_steps=10000)
        assert rel_err(g["x"][r:r + 1], o["x"]).max() <= 1e-5
        assert rel_err(g["y"][r:r + 1], o["y"]).max() <= 1e-5


@pytest.mark.parametrize("plan", ["fp32", "mixed"])
def test_gaussian_bsb_and_fp64_energies(plan):
    J = synth.gaussian_instance(300, 3)
    say("gaussian bsb", plan)
    c0 = 0.5  # c1 / (sigma_J sqrt(N)) with sigma_J = 1/sqrt(N)
    g = gpu_run(J, hsb.HSB_BSB, plan, 50, 32, c0=c0, gamma=0.01, schedule_steps=1000)
    o = oracle_run(J, oracle.BSB, oracle.FP64, 50, 32, c0=c0, gamma=0.01, schedule_steps=1000)
    assert g["last_plan"] == ("digits" if plan == "mixed" else "fp32")
    assert rel_err(g["x"], o["x"]).max() <= 1e-5 and rel_err(g["y"], o["y"]).max() <= 1e-5
    g = gpu_run(J, hsb.HSB_BSB, plan, 1000, 32, c0=c0, gamma=0.01)
    for s, e in zip(g["spins"], g["energy"]):
        ref = oracle.energy(J, s)
        assert abs(e - ref) <= 1e-12 * abs(ref)


def test_gaussian_full_size_bsb_digits():
    """N=2000 Gaussian couplings (four-digit J), R=1024, first 50 steps of 10^4."""
    J = synth.gaussian_instance(2000, 3)
    say("gaussian full size digits")
    g = gpu_run(J, hsb.HSB_BSB, "mixed", 50, 1024, seed=4, c0=0.5, gamma=0.01,
                schedule_steps=10000)
    assert g["last_plan"] == "digits"
    for r in (0, 333, 1023):
        o = oracle_run(J, oracle.BSB, oracle.FP64, 50, 1, seed=4, c0=0.5, gamma=0.01, r0=r,
                       schedule_steps=10000)
        assert rel_err(g["x"][r:r + 1], o["x"]).max() <= 1e-5
        assert rel_err(g["y"][r:r + 1], o["y"]).max() <= 1e-5


@pytest.mark.parametrize("scale", [1, 5])
def test_bsb_mixed_deterministic_prefix_and_resume(scale):
    J, c0, expect = bsb_case("mixed", scale, 300, 6)
    R, Ns, k = 48, 400, 150
    say("bsb mixed determinism", expect)
    a = gpu_run(J, hsb.HSB_BSB, "mixed", Ns, R, c0=c0, gamma=0.02, seed=9)
    assert a["last_plan"] == expect
    b = gpu_run(J, hsb.HSB_BSB, "mixed", Ns, R, c0=c0, gamma=0.02, seed=9)
    d = gpu_run(J, hsb.HSB_BSB, "mixed", Ns, 17, c0=c0, gamma=0.02, seed=9)
    for key in ("x", "y", "spins", "energy", "best_step"):
        assert np.array_equal(a[key], b[key]), key
    assert np.array_equal(d["x"], a["x"][:17]) and np.array_equal(d["energy"], a["energy"][:17])
    h1 = gpu_run(J, hsb.HSB_BSB, "mixed", k, R, c0=c0, gamma=0.02, seed=9, schedule_steps=Ns)
    h2 = gpu_run(J, hsb.HSB_BSB, "mixed", Ns - k, R, c0=c0, gamma=0.02, start_step=k,
                 schedule_steps=Ns, x0=torch.from_numpy(h1["x"]), y0=torch.from_numpy(h1["y"]))
    assert np.array_equal(h2["x"], a["x"]) and np.array_equal(h2["y"], a["y"])
    # energies are eq. (1) of the returned spins, exactly
    for s_, e in zip(a["spins"], a["energy"]):
        assert oracle.energy(J, s_) == e


@pytest.mark.parametrize("N,R,steps,interval", [(1, 3, 40, 7), (63, 33, 60, 25),
                                                (65, 64, 50, 50), (257, 40, 50, 1),
                                                (700, 96, 50, 20)])
def test_bsb_fp4_ragged_shapes(N, R, steps, interval):
    """bSB on the FP4 plan at ragged sizes: the 1e-5 bar over the first steps of a
    2000-step schedule, and energies equal to eq. (1) of the returned spins."""
    J = synth.sk_instance(N, N + 5)
    c0 = 0.5 / np.sqrt(N)
    say("bsb fp4 ragged", N, R, steps, interval)
    g = gpu_run(J, hsb.HSB_BSB, "mixed", steps, R, seed=N, c0=c0, gamma=0.01, interval=interval,
                schedule_steps=2000)
    assert g["last_plan"] == "fp4"
    o = oracle_run(J, oracle.BSB, oracle.FP64, steps, R, seed=N, c0=c0, gamma=0.01,
                   interval=interval, schedule_steps=2000)
    assert rel_err(g["x"], o["x"]).max() <= 1e-5 and rel_err(g["y"], o["y"]).max() <= 1e-5
    for s_, e in zip(g["spins"], g["energy"]):
        assert oracle.energy(J, s_) == e


@pytest.mark.parametrize("steps", [1, 20])
def test_bsb_fp4_chunk_scales_differ(steps):
    """bSB on the FP4 plan from a start state whose 32-row chunks differ in
    magnitude by factors of 2 up to 2^7, so that the digits' block scales change
    from every K block to the next (in the usual start states they are nearly
    all equal): a product that used another block's scale would miss the 1e-5
    bar.  Also the bar on y."""
    N, R = 512, 64
    J = synth.sk_instance(N, 31)
    c0 = 0.5 / np.sqrt(N)
    x0, y0 = oracle.init_state(9, R, N, amp=0.9)
    scale = (2.0 ** -((np.arange(N) // 32) % 8)).astype(np.float32)
    x0 = (x0 * scale).astype(np.float32)
    y0 = (y0 * scale * np.float32(0.1)).astype(np.float32)
    say("bsb fp4 chunk scales", steps)
    g = gpu_run(J, hsb.HSB_BSB, "mixed", steps, R, c0=c0, gamma=0.01, schedule_steps=2000,
                x0=torch.from_numpy(x0), y0=torch.from_numpy(y0))
    assert g["last_plan"] == "fp4"
    o = oracle_run(J, oracle.BSB, oracle.FP64, steps, R, c0=c0, gamma=0.01, schedule_steps=2000,
                   x0=x0, y0=y0)
    assert rel_err(g["x"], o["x"]).max() <= 1e-5
    assert rel_err(g["y"], o["y"]).max() <= 1e-5


def test_dsb_real_j_digits_and_host_api():
    """dSB on Gaussian couplings with the digit plan (four-digit J): the early
    trajectory within the 1e-5 bar of FP64; the host-buffer entry point returns
    the same spins and energies as the device one."""
    J = synth.gaussian_instance(300, 8)
    say("dsb real J digits")
    g = gpu_run(J, hsb.HSB_DSB, "mixed", 50, 16, c0=0.5, gamma=0.01, schedule_steps=1000)
    assert g["last_plan"] == "digits"
    o = oracle_run(J, oracle.DSB, oracle.FP64, 50, 16, c0=0.5, gamma=0.01, schedule_steps=1000)
    assert rel_err(g["x"], o["x"]).max() <= 1e-5 and rel_err(g["y"], o["y"]).max() <= 1e-5
    with hsb.Context(J, precision="mixed", init_amp=0.1) as ctx:
        spins, energy, rc = ctx.run(hsb.HSB_DSB, 1.0, 0.5, 1.0, 0.01, 200, 16, 3)
        dev = ctx.run_ex(hsb.HSB_DSB, 200, 16, 1.0, 0.5, 1.0, 0.01, 3)
        torch.cuda.synchronize()
    assert rc == hsb.HSB_OK
    assert np.array_equal(spins, dev["spins"].cpu().numpy())
    assert np.array_equal(energy, dev["energy"].cpu().numpy())
    for s_, e in zip(spins, energy):
        ref = oracle.energy(J, s_)
        assert abs(e - ref) <= 1e-12 * abs(ref)


def test_bsb_digits_need_bounded_start_state():
    J = synth.sk_instance(64, 2)
    say("bsb digits start-state bound")
    with pytest.raises(hsb.HSBError) as ei:
        gpu_run(J, hsb.HSB_BSB, "mixed", 10, 8, amp=1.5)
    assert ei.value.code == hsb.HSB_EUNSUPPORTED
    g = gpu_run(J, hsb.HSB_BSB, "auto", 10, 8, amp=1.5)
    assert g["last_plan"] == "fp32"
    f = gpu_run(J, hsb.HSB_BSB, "fp32", 10, 8, amp=1.5)
    assert np.array_equal(g["x"], f["x"])


# ---------------------------------------------------------------- errors

def test_plan_selection_and_unsupported():
    say("plans")
    with hsb.Context(synth.sk_instance(64, 1)) as ctx:
        assert ctx.plan(hsb.HSB_DSB) == "mixed" and ctx.plan(hsb.HSB_BSB) == "mixed"
    with hsb.Context(synth.gaussian_instance(64, 1)) as ctx:
        assert ctx.plan(hsb.HSB_DSB) == "fp32" and ctx.plan(hsb.HSB_BSB) == "mixed"
    with hsb.Context(synth.gaussian_instance(64, 1), precision="mixed") as ctx:
        assert ctx.plan(hsb.HSB_DSB) == "mixed"


@pytest.mark.parametrize("variant,plan", [(1, "fp32"), (1, "mixed"), (0, "mixed")])
def test_non_finite_state_is_reported(variant, plan):
    """gamma*dt > 1 with walls: y grows geometrically (eq. (22)) until it overflows."""
    J = synth.sk_instance(40, 1)
    say("numeric", variant, plan)
    g = gpu_run(J, variant, plan, 400, 8, gamma=8.0, dt=1.0, allow_numeric=True)
    assert g["status"] == hsb.HSB_ENUMERIC
    assert np.all(np.isnan(g["energy"]))


def test_invalid_run_arguments():
    J = synth.sk_instance(16, 1)
    say("invalid args")
    with hsb.Context(J) as ctx:
        for kw in (dict(steps=-1), dict(R=0), dict(dt=0.0), dict(gamma=-0.1),
                   dict(dt=float("nan")), dict(schedule_steps=5)):
            args = dict(variant=hsb.HSB_DSB, steps=10, R=4, a0=1.0, c0=0.1, dt=1.0, gamma=0.0)
            args.update(kw)
            with pytest.raises(hsb.HSBError) as ei:
                ctx.run_ex(args.pop("variant"), args.pop("steps"), args.pop("R"), args.pop("a0"),
                           args.pop("c0"), args.pop("dt"), args.pop("gamma"), **args)
            assert ei.value.code == hsb.HSB_EINVAL
