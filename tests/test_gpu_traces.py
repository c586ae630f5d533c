"""Per-sample traces of hsb_run_ex (marked `gpu`): the energy (eq. (1)) and
the instantaneous temperature T_inst = (1/N) sum_i y_i^2 (eq. (9)) of every
sample point, on every plan, through the C ABI, against the oracle's traces.

Bars:
  - dSB: the state is bitwise the oracle's FP32 mirror, so the energies are
    equal and T_inst (FP64 sums of exact squares, another order) agrees to
    1e-13 relative.
  - bSB: every trace row is eq. (1) / eq. (9) of the state at that sample
    point (obtained by resumed calls); where that state is within the 1e-5
    bar of the FP64 oracle's, T_inst is within (1 + 1e-5)^2 - 1 < 2.1e-5
    relative of the oracle's, and equal spins give equal energies.  A wall
    event taken on one side only puts a replica outside the bar (counted).
  - at the bench configuration (N = 2000, R = 1024, 10^4 steps, FP4 plan):
    the last row is the final energy, the row minimum the best energy, and its
    earliest row the best step.
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


def gpu_traces(J, variant, plan, steps, R, interval, seed=1, gamma=0.01, start_step=0,
               schedule_steps=0, x0=None, y0=None, expect_plan=None):
    N = J.shape[0]
    with hsb.Context(J, precision=plan, init_amp=0.1, energy_interval=interval) as ctx:
        out = ctx.run_ex(variant, steps, R, 1.0, 0.5 / np.sqrt(N), 1.0, gamma, seed, traces=True,
                         want_state=True, start_step=start_step, schedule_steps=schedule_steps,
                         x0=x0, y0=y0)
        torch.cuda.synchronize()
        if expect_plan:
            assert ctx.last_plan() == expect_plan
        assert ctx.num_samples(start_step, steps) == out["trace_energy"].shape[0]
        return {k: v.cpu().numpy() for k, v in out.items() if hasattr(v, "cpu")}


def oracle_traces(J, variant, precision, steps, R, interval, seed=1, gamma=0.01, **kw):
    N = J.shape[0]
    return oracle.run(J, variant, 1.0, np.float32(0.5 / np.sqrt(N)), 1.0, gamma, steps, R,
                      seed=seed, amp=0.1, interval=interval, precision=precision, traces=True,
                      **kw)


def assert_consistent(g):
    """The traces agree with the run's own outputs (any plan, any size)."""
    te = g["trace_energy"]
    assert np.array_equal(te[-1], g["final_energy"])
    assert np.array_equal(te.min(axis=0), g["best_energy"])
    assert np.all(np.isfinite(g["trace_tinst"])) and np.all(g["trace_tinst"] >= 0)


@pytest.mark.parametrize("plan,expect", [("fp32", "fp32"), ("mixed", "fp4"),
                                         ("digits", "digits")])
@pytest.mark.parametrize("N,R,steps,interval", [(300, 40, 250, 50), (130, 33, 250, 60),
                                                (65, 7, 0, 10)])
def test_dsb_traces_equal_mirror(plan, expect, N, R, steps, interval):
    J = synth.sk_instance(N, 31)
    say("dsb traces", plan, N, R, steps, interval)
    g = gpu_traces(J, hsb.HSB_DSB, plan, steps, R, interval, expect_plan=expect)
    o = oracle_traces(J, oracle.DSB, oracle.FP32, steps, R, interval)
    assert g["trace_energy"].shape == o["trace_e"].shape == (oracle.num_samples(steps, interval), R)
    assert np.array_equal(g["trace_energy"], o["trace_e"])
    np.testing.assert_allclose(g["trace_tinst"], o["trace_tinst"], rtol=1e-13, atol=0)
    assert_consistent(g)


@pytest.mark.parametrize("plan", ["fp32", "mixed", "digits"])
def test_dsb_split_run_traces_concatenate(plan):
    """Two calls (0..130, 130..250; interval 50) against one call (0..250):
    the first call's last row is the extra sample at step 130, the other rows
    are the one call's rows in order."""
    N, R = 200, 24
    J = synth.sk_instance(N, 32)
    say("dsb split traces", plan)
    one = gpu_traces(J, hsb.HSB_DSB, plan, 250, R, 50)
    a = gpu_traces(J, hsb.HSB_DSB, plan, 130, R, 50, schedule_steps=250)
    b = gpu_traces(J, hsb.HSB_DSB, plan, 120, R, 50, start_step=130, schedule_steps=250,
                   x0=torch.from_numpy(a["x"]).cuda(), y0=torch.from_numpy(a["y"]).cuda())
    assert a["trace_energy"].shape[0] == 3 and b["trace_energy"].shape[0] == 3
    for k in ("trace_energy", "trace_tinst"):
        assert np.array_equal(np.concatenate([a[k][:2], b[k]]), one[k])


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


@pytest.mark.parametrize("plan,expect", [("fp32", "fp32"), ("mixed", "fp4"),
                                         ("digits", "digits")])
def test_bsb_traces_are_those_of_the_sampled_states(plan, expect):
    """bSB, 50 steps sampled every 10: chained calls of 10 steps (resume) give
    the state at every sample point.  Each trace row is eq. (1) of sgn(x) and
    eq. (9) of y of that state, and the chained rows are the single call's.
    Against the FP64 oracle (its states after 10, 20, .. 50 steps): wherever a
    replica's x and y are within the 1e-5 bar, T_inst is within 2.1e-5, and
    equal spins give the same energy.  Replicas outside the bar (a wall event
    on one side only) are counted."""
    N, R, I, n = 300, 48, 10, 5
    J = synth.sk_instance(N, 33)
    J64 = J.astype(np.float64)
    say("bsb traces", plan)
    one = gpu_traces(J, hsb.HSB_BSB, plan, n * I, R, I, expect_plan=expect)
    assert one["trace_energy"].shape == (n, R)
    assert_consistent(one)
    x = y = None
    inside = 0
    for c in range(n):
        g = gpu_traces(J, hsb.HSB_BSB, plan, I, R, I, start_step=c * I, schedule_steps=n * I,
                       x0=x, y0=y)
        assert g["trace_energy"].shape == (1, R)
        s = np.where(g["x"] >= 0, 1.0, -1.0)
        e_def = -0.5 * np.einsum("ri,ij,rj->r", s, J64, s)
        t_def = (g["y"].astype(np.float64) ** 2).sum(axis=1) / N
        assert np.array_equal(g["trace_energy"][0], e_def)
        np.testing.assert_allclose(g["trace_tinst"][0], t_def, rtol=1e-13, atol=0)
        assert np.array_equal(g["trace_energy"][0], one["trace_energy"][c])
        assert np.array_equal(g["trace_tinst"][0], one["trace_tinst"][c])
        o = oracle_traces(J, oracle.BSB, oracle.FP64, (c + 1) * I, R, I, schedule_steps=n * I)
        ok = (rel_err(g["x"], o["x"]) <= 1e-5) & (rel_err(g["y"], o["y"]) <= 1e-5)
        inside += int(ok.sum())
        np.testing.assert_allclose(g["trace_tinst"][0][ok], o["trace_tinst"][-1][ok],
                                   rtol=2.1e-5, atol=0)
        same = np.all(np.where(o["x"] >= 0, 1.0, -1.0) == s, axis=1)
        assert np.array_equal(g["trace_energy"][0][same], o["trace_e"][-1][same])
        x, y = torch.from_numpy(g["x"]).cuda(), torch.from_numpy(g["y"]).cuda()
    say(f"replica-samples within the 1e-5 bar: {inside} of {n * R}")
    assert inside >= n * R // 2


def test_gaussian_traces_fp64_energies():
    """Real J on the digit plan: FP64 energies of the same spins agree to 1e-12
    wherever the spins are the same (nearly everywhere after 20 steps)."""
    N, R, steps, interval = 257, 20, 20, 5
    J = synth.gaussian_instance(N, 34)
    say("gaussian traces")
    with hsb.Context(J, precision="digits", init_amp=0.1, energy_interval=interval) as ctx:
        out = ctx.run_ex(hsb.HSB_BSB, steps, R, 1.0, 0.5, 1.0, 0.01, 1, traces=True)
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in out.items() if hasattr(v, "cpu")}
    o = oracle.run(J, oracle.BSB, 1.0, np.float32(0.5), 1.0, 0.01, steps, R, seed=1, amp=0.1,
                   interval=interval, precision=oracle.FP64, traces=True)
    rel = np.abs(g["trace_energy"] - o["trace_e"]) / np.abs(o["trace_e"])
    assert np.mean(rel <= 1e-12) >= 0.99
    np.testing.assert_allclose(g["trace_tinst"], o["trace_tinst"], rtol=2.1e-5, atol=0)
    assert_consistent(g)


@pytest.mark.parametrize("variant", [hsb.HSB_DSB, hsb.HSB_BSB])
def test_traces_at_bench_configuration(variant):
    """N = 2000, R = 1024, 10^4 steps, interval 100 on the FP4 plan: 100 rows
    consistent with the run's outputs; the best step is the earliest row at the
    minimum; a trace run changes nothing else (outputs equal a run without)."""
    N, R, steps = 2000, 1024, 10000
    J = synth.sk_instance(N, 2000)
    say("bench-size traces", variant)
    c0 = 0.5 / np.sqrt(N)
    with hsb.Context(J, precision="mixed", energy_interval=100) as ctx:
        g = ctx.run_ex(variant, steps, R, 1.0, c0, 1.0, 0.01, 7, traces=True)
        plain = ctx.run_ex(variant, steps, R, 1.0, c0, 1.0, 0.01, 7)
        torch.cuda.synchronize()
        assert ctx.last_plan() == "fp4"
        g = {k: v.cpu().numpy() for k, v in g.items() if hasattr(v, "cpu")}
        plain = {k: v.cpu().numpy() for k, v in plain.items() if hasattr(v, "cpu")}
    assert g["trace_energy"].shape == (100, R)
    assert_consistent(g)
    first_min = np.argmax(g["trace_energy"] == g["best_energy"][None, :], axis=0)
    assert np.array_equal((first_min + 1) * 100, g["best_step"])
    for k in ("spins", "energy", "best_energy", "final_energy", "best_step"):
        assert np.array_equal(g[k], plain[k]), k
    say("median T_inst at samples 1, 50, 100:", np.median(g["trace_tinst"][[0, 49, 99]], axis=1))


def test_trace_runs_are_graph_launched_identically():
    """A repeated FP4 dSB run with traces is launched as a graph and gives the
    eager traces each time."""
    N, R = 500, 64
    J = synth.sk_instance(N, 35)
    say("graph traces")
    c0 = 0.5 / np.sqrt(N)
    with hsb.Context(J, precision="mixed", energy_interval=40) as ctx:
        dev = torch.device("cuda", 0)
        ns = ctx.num_samples(0, 300)
        o = {"trace_energy": torch.empty((ns, R), dtype=torch.float64, device=dev),
             "trace_tinst": torch.empty((ns, R), dtype=torch.float64, device=dev),
             "spins": torch.empty((R, N), dtype=torch.int8, device=dev)}
        for k in ("energy", "best_energy", "final_energy"):
            o[k] = torch.empty(R, dtype=torch.float64, device=dev)
        o["best_step"] = torch.empty(R, dtype=torch.int32, device=dev)
        ref = None
        for i in range(4):
            for t in o.values():
                t.fill_(3)
            ctx.run_ex(hsb.HSB_DSB, 300, R, 1.0, c0, 1.0, 0.01, 5, traces=True, out=o)
            torch.cuda.synchronize()
            got = {k: o[k].cpu().numpy().copy() for k in ("trace_energy", "trace_tinst")}
            if ref is None:
                ref = got
            for k in got:
                assert np.array_equal(got[k], ref[k]), (i, k)
        assert ctx.get_option("graph_launches") == 3
    orc = oracle_traces(J, oracle.DSB, oracle.FP32, 300, R, 40, seed=5)
    assert np.array_equal(ref["trace_energy"], orc["trace_e"])
