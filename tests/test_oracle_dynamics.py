"""Pins for the oracle's time stepping (Methods, eqs. (16)-(22)) and its runs.

What fixes each part independently of the oracle's code:
  - hand-worked single steps (tests/golden/step_cases.json);
  - convergence, at first order in dt, to an independent ODE solution (scipy)
    of the heated equations of motion, eqs. (10)-(11), with the linear pump;
  - the kick-then-drift structure and symplecticity (unit determinant) of the
    unheated, wall-free step;
  - invariants: |x| <= 1 after every step, a wall hit leaves y' = gamma dt y;
  - exact global-flip and gauge symmetry of whole trajectories;
  - brute-force ground states bound (and are reached by) the sampled energies;
  - the Nose-Hoover thermostat (eqs. (6)-(8)): heated SB at infinite mass, an
    independent loop of its recursion for free particles, and the change of
    xi over a run against the T_inst traces of the states before each step.
"""
import json
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import synth


def _cases(golden_dir):
    with open(os.path.join(golden_dir, "step_cases.json")) as fh:
        return json.load(fh)["cases"]


@pytest.mark.parametrize("precision", [oracle.FP64, oracle.FP32])
def test_hand_worked_steps(golden_dir, precision):
    for c in _cases(golden_dir):
        J = np.array(c["J"], dtype=np.float64)
        f = oracle.field(J, np.array(c["x"], dtype=np.float64), c["variant"])
        x, y = oracle.update(f, c["x"], c["y"], c["p"], c["a0"], c["c0"], c["dt"], c["gamma"],
                             precision)
        assert np.array_equal(np.asarray(x, dtype=np.float64), c["x_new"]), c["name"]
        assert np.array_equal(np.asarray(y, dtype=np.float64), c["y_new"]), c["name"]


def test_run_reproduces_hand_worked_first_step(golden_dir):
    # the run driver uses p = a0 - a(t_0) = a0 at the first step
    c = [c for c in _cases(golden_dir) if c["p"] == 1.0 and c["variant"] == 1][0]
    r = oracle.run(np.array(c["J"]), c["variant"], c["a0"], c["c0"], c["dt"], c["gamma"],
                   steps=1, R=1, x0=np.array([c["x"]]), y0=np.array([c["y"]]))
    assert np.array_equal(r["x"][0], c["x_new"]) and np.array_equal(r["y"][0], c["y_new"])


@pytest.mark.parametrize("gamma", [0.0, 0.3])
def test_converges_to_ode_first_order(gamma):
    """Without walls the discrete map is a first-order integrator of eqs. (10)-(11)."""
    N, a0, c0, T = 4, 1.0, 0.2, 4.0
    J = synth.sk_instance(N, 3).astype(np.float64)
    x0, y0 = oracle.init_state(9, 1, N, amp=0.05)

    def rhs(t, z):
        x, y = z[:N], z[N:]
        return np.concatenate([a0 * y, -(a0 - a0 * t / T) * x + c0 * (J @ x) + gamma * y])

    sol = solve_ivp(rhs, (0, T), np.concatenate([x0[0], y0[0]]).astype(np.float64),
                    method="DOP853", rtol=1e-12, atol=1e-14, dense_output=True)
    assert np.abs(sol.sol(np.linspace(0, T, 400))[:N]).max() < 0.9  # walls never touched
    errs = []
    for dt in (0.01, 0.005, 0.0025):
        r = oracle.run(J, oracle.BSB, a0, c0, dt, gamma, int(round(T / dt)), 1, x0=x0, y0=y0)
        errs.append(np.abs(np.concatenate([r["x"][0], r["y"][0]]) - sol.y[:, -1]).max())
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    assert all(1.8 < q < 2.2 for q in ratios), (errs, ratios)
    assert errs[-1] < 1e-3


def test_step_is_kick_then_drift_and_symplectic():
    """gamma = 0, no coupling, no wall: the step is linear with det 1 (symplectic Euler).

    Kick first (y from the old x) then drift (x from the new y) makes dy'/dy = 1
    and dx'/dy = a0 dt, distinguishing it from drift-then-kick.
    """
    f = np.zeros(1)
    for p, a0, dt in [(0.7, 1.0, 0.5), (0.3, 1.3, 0.9)]:
        ex = oracle.update(f, [0.25], [0.0], p, a0, 0.5, dt, 0.0)
        ey = oracle.update(f, [0.0], [0.25], p, a0, 0.5, dt, 0.0)
        M = np.array([[ex[0][0], ey[0][0]], [ex[1][0], ey[1][0]]]) / 0.25
        assert np.linalg.det(M) == pytest.approx(1.0, abs=1e-14)
        assert M[1, 1] == 1.0 and M[0, 1] == pytest.approx(a0 * dt, rel=1e-15)
        assert M[1, 0] == pytest.approx(-p * dt, rel=1e-15)


@pytest.mark.parametrize("precision", [oracle.FP64, oracle.FP32])
@pytest.mark.parametrize("variant", [oracle.BSB, oracle.DSB])
def test_wall_invariants(precision, variant):
    N, gamma, dt = 24, 0.2, 1.5
    J = synth.sk_instance(N, 5)
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, N)
    y = rng.uniform(-2, 2, N)
    if precision == oracle.FP32:
        x, y = x.astype(np.float32), y.astype(np.float32)
    walls = 0
    for k in range(200):
        f = oracle.field(J, np.asarray(x, dtype=np.float64), variant)
        xn, yn = oracle.update(f, x, y, 1.0 - k / 200, 1.0, 0.3, dt, gamma, precision)
        assert np.all(np.abs(xn) <= 1.0)
        hit = np.abs(xn) == 1.0
        walls += int(hit.sum())
        if precision == oracle.FP64:
            assert np.allclose(yn[hit], gamma * dt * np.asarray(y)[hit], rtol=1e-15, atol=0)
        else:
            gdt = np.float32(np.float32(gamma) * np.float32(dt))
            assert np.array_equal(yn[hit], (gdt * np.asarray(y)[hit]).astype(np.float32))
        x, y = xn, yn
    assert walls > 100  # the invariant was exercised


@pytest.mark.parametrize("precision", [oracle.FP64, oracle.FP32])
@pytest.mark.parametrize("variant", [oracle.BSB, oracle.DSB])
def test_global_flip_and_gauge_symmetry(precision, variant):
    N, R, steps = 30, 4, 300
    J = synth.sk_instance(N, 8)
    x0, y0 = oracle.init_state(21, R, N)
    kw = dict(variant=variant, a0=1.0, c0=0.5 / np.sqrt(N), dt=0.9, gamma=0.05, steps=steps,
              R=R, precision=precision, interval=50)
    base = oracle.run(J, x0=x0, y0=y0, **kw)
    flip = oracle.run(J, x0=-x0, y0=-y0, **kw)
    assert np.array_equal(flip["x"], -base["x"]) and np.array_equal(flip["y"], -base["y"])
    assert np.array_equal(flip["best_e"], base["best_e"])
    d = np.where(np.random.default_rng(2).random(N) < 0.5, -1, 1).astype(np.float32)
    Jg = d[:, None] * J * d[None, :]
    gauge = oracle.run(Jg, x0=x0 * d, y0=y0 * d, **kw)
    assert np.array_equal(gauge["x"], base["x"] * d) and np.array_equal(gauge["y"], base["y"] * d)
    assert np.array_equal(gauge["best_e"], base["best_e"])
    assert np.array_equal(gauge["spins"], (base["spins"] * d).astype(np.int8))


@pytest.mark.parametrize("variant,gamma,dt", [(oracle.BSB, 0.5, 1.1), (oracle.DSB, 0.06, 1.1),
                                              (oracle.BSB, 0.0, 0.7), (oracle.DSB, 0.0, 1.1)])
def test_runs_bounded_by_and_reach_ground_state(variant, gamma, dt):
    N = 14
    J = synth.sk_instance(N, 11)
    emin = oracle.brute_force(J)[0]
    r = oracle.run(J, variant, 1.0, 0.5 / np.sqrt(N), dt, gamma, 1000, 64, seed=5)
    assert np.all(r["best_e"] >= emin)
    assert np.all(r["best_e"] <= r["final_e"])
    assert np.mean(r["best_e"] == emin) > 0.2
    for s, e in zip(r["spins"], r["energy"]):
        assert oracle.energy(J, s) == e


def test_sampling_schedule_and_traces():
    N, R = 20, 3
    J = synth.sk_instance(N, 2)
    assert oracle.num_samples(0, 100) == 1
    assert oracle.num_samples(100, 100) == 1
    assert oracle.num_samples(250, 100) == 3
    r = oracle.run(J, oracle.DSB, 1.0, 0.1, 1.0, 0.01, 250, R, seed=1, traces=True)
    te = r["trace_e"]
    assert te.shape == (3, R)
    assert np.array_equal(te[-1], r["final_e"]) and np.array_equal(te.min(0), r["best_e"])
    assert np.allclose(r["trace_tinst"][-1], (r["y"] ** 2).mean(1), rtol=1e-14)  # eq. (9)
    assert set(r["best_step"]) <= {100, 200, 250}
    # interval = Ns evaluates only the last state (700-spin protocol)
    r2 = oracle.run(J, oracle.DSB, 1.0, 0.1, 1.0, 0.01, 250, R, seed=1, interval=250)
    assert np.array_equal(r2["best_e"], r2["final_e"]) and np.array_equal(r2["final_e"],
                                                                            r["final_e"])
    # return_best=False returns the final spins
    r3 = oracle.run(J, oracle.DSB, 1.0, 0.1, 1.0, 0.01, 250, R, seed=1, return_best=False)
    assert np.array_equal(r3["energy"], r["final_e"])
    assert np.array_equal(r3["spins"], np.where(r3["x"] >= 0, 1, -1))


def test_zero_steps_samples_initial_state():
    J = synth.sk_instance(10, 2)
    r = oracle.run(J, oracle.BSB, 1.0, 0.1, 1.0, 0.0, 0, 2, seed=4)
    x0, _ = oracle.init_state(4, 2, 10)
    assert np.array_equal(r["x"], x0.astype(np.float64))
    assert np.array_equal(r["spins"], np.where(x0 >= 0, 1, -1))


def test_replica_independence_and_per_replica_gamma():
    N = 25
    J = synth.sk_instance(N, 6)
    full = oracle.run(J, oracle.DSB, 1.0, 0.1, 1.0, 0.02, 120, 6, seed=3)
    part = oracle.run(J, oracle.DSB, 1.0, 0.1, 1.0, 0.02, 120, 2, seed=3, r0=3)
    assert np.array_equal(full["x"][3:5], part["x"]) and np.array_equal(full["y"][3:5], part["y"])
    g = np.array([0.02, 0.0, 0.02, 0.02, 0.0, 0.02])
    mixed = oracle.run(J, oracle.DSB, 1.0, 0.1, 1.0, g, 120, 6, seed=3)
    zero = oracle.run(J, oracle.DSB, 1.0, 0.1, 1.0, 0.0, 120, 6, seed=3)
    assert np.array_equal(mixed["x"][g > 0], full["x"][g > 0])
    assert np.array_equal(mixed["x"][g == 0], zero["x"][g == 0])


def test_fp32_mirror_tracks_fp64_short_run():
    N = 60
    J = synth.sk_instance(N, 4)
    kw = dict(variant=oracle.BSB, a0=1.0, c0=0.5 / np.sqrt(N), dt=0.5, gamma=0.01, steps=20, R=4,
              seed=8)
    a = oracle.run(J, precision=oracle.FP64, **kw)
    b = oracle.run(J, precision=oracle.FP32, **kw)
    rel = np.linalg.norm(a["x"] - b["x"], axis=1) / np.linalg.norm(a["x"], axis=1)
    assert rel.max() < 1e-5


def test_step_to_solution_eq15():
    assert oracle.step_to_solution(0.0, 1000) == np.inf
    assert oracle.step_to_solution(0.5, 1000) == pytest.approx(6643.856189774724, rel=1e-12)
    assert oracle.step_to_solution(0.995, 1000) == 1000.0


# ---------------------------------------------------------------- eqs. (6)-(8)

@pytest.mark.parametrize("precision", [oracle.FP64, oracle.FP32])
@pytest.mark.parametrize("variant", [oracle.BSB, oracle.DSB])
def test_nose_hoover_with_infinite_mass_is_heated_sb(precision, variant):
    """1/M = 0 keeps xi at its start value -gamma: the heated SB of eqs.
    (10)-(11) is the thermostat with a constant xi, bit for bit."""
    J = synth.sk_instance(40, 5)
    kw = dict(seed=3, amp=0.5, interval=25, precision=precision, traces=True)
    heated = oracle.run(J, variant, 1.0, 0.08, 0.9, 0.07, 300, 6, **kw)
    nh = oracle.run(J, variant, 1.0, 0.08, 0.9, 0.07, 300, 6, nose_hoover=(0.0, 0.4), **kw)
    for k in ("x", "y", "best_e", "final_e", "best_step", "trace_e", "trace_tinst"):
        assert np.array_equal(heated[k], nh[k]), k
    # the FP32 mirror's gamma is a float
    assert np.all(nh["xi"] == (-0.07 if precision == oracle.FP64 else -float(np.float32(0.07))))


def test_nose_hoover_free_particles_follow_the_recursion():
    """J = 0 and a0 = 0: x stays put and eqs. (7)-(8) leave
    y(t_k+1) = y(t_k) - xi(t_k) y(t_k) dt,
    xi(t_k+1) = xi(t_k) + (dt/M) (sum_i y_i(t_k)^2 - N T),
    computed here by an independent loop.  Started below the temperature T,
    xi turns negative and T_inst rises (the heating described after eq. (9))."""
    N, R, K, dt, inv_m, T = 5, 3, 40, 0.5, 0.2, 0.3
    J = np.zeros((N, N))
    rng = np.random.default_rng(1)
    x0 = rng.uniform(-0.5, 0.5, (R, N))
    y0 = rng.uniform(-0.2, 0.2, (R, N))  # T_inst(0) <= 0.04 < T
    xi0 = np.array([0.0, 0.1, -0.05])
    o = oracle.run(J, oracle.BSB, 0.0, 0.3, dt, 0.0, K, R, x0=x0, y0=y0, nose_hoover=(inv_m, T),
                   xi0=xi0, precision=oracle.FP64)
    y = y0.astype(np.float32).astype(np.float64)
    xi = xi0.copy()
    xis = [xi.copy()]
    for _ in range(K):
        s = (y * y).sum(axis=1)
        y = y - xi[:, None] * y * dt
        xi = xi + dt * inv_m * (s - N * T)
        xis.append(xi.copy())
    np.testing.assert_allclose(o["y"], y, rtol=1e-12)
    np.testing.assert_allclose(o["xi"], xi, rtol=1e-12, atol=1e-15)
    assert np.array_equal(o["x"], x0.astype(np.float32).astype(np.float64))
    assert np.all(np.array(xis)[1] < xi0) and np.all(np.array(xis)[5] < 0)
    # while T_inst < T the thermostat heats: T_inst after 6 steps is larger
    early = oracle.run(J, oracle.BSB, 0.0, 0.3, dt, 0.0, 6, R, x0=x0, y0=y0,
                       nose_hoover=(inv_m, T), xi0=xi0, precision=oracle.FP64)
    t0 = (y0.astype(np.float32).astype(np.float64) ** 2).mean(axis=1)
    assert np.all((early["y"] ** 2).mean(axis=1) > t0)


@pytest.mark.parametrize("variant", [oracle.BSB, oracle.DSB])
def test_nose_hoover_xi_integrates_the_states_before_each_step(variant):
    """Summed over K steps, eq. (8) gives xi(t_K) - xi(t_0) = (dt/M) sum over
    k = 0 .. K-1 of (N T_inst(t_k) - N T): the T_inst traces of the states
    after 0 .. K-1 steps (not 1 .. K) account for the change of xi."""
    N, R, K, dt, inv_m, T = 60, 4, 120, 0.8, 0.01, 0.05
    J = synth.sk_instance(N, 9)
    kw = dict(seed=4, amp=0.6, precision=oracle.FP64, nose_hoover=(inv_m, T))
    first = oracle.run(J, variant, 1.0, 0.1, dt, 0.02, 0, R, interval=1, traces=True, **kw)
    o = oracle.run(J, variant, 1.0, 0.1, dt, 0.02, K, R, interval=1, traces=True, **kw)
    tinst = np.concatenate([first["trace_tinst"], o["trace_tinst"]])  # states 0 .. K
    want = -0.02 + dt * inv_m * (N * tinst[:K] - N * T).sum(axis=0)
    np.testing.assert_allclose(o["xi"], want, rtol=1e-10)
    wrong = -0.02 + dt * inv_m * (N * tinst[1:] - N * T).sum(axis=0)
    assert not np.allclose(o["xi"], wrong, rtol=1e-6)
