"""Graph launches of repeated runs (HSB_OPT_GRAPH) through the C ABI.

dSB on the FP4 plan: the first call with given arguments runs eagerly, the
next identical call captures its queued work into a HIP graph, and later
identical calls launch that graph (the seed is read when it runs, so calls
that differ only in the seed share it).  Every launch must give exactly the
eager run's outputs, with other eager GPU work and synchronisations in
between, and any other run on the context must drop the graph.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_08361_amd import hsb  # noqa: E402

KEYS = ("spins", "energy", "best_energy", "final_energy", "best_step", "x", "y")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    hsb.load_library()


def say(*a):
    print("[case]", *a, flush=True)


def outputs(R, N):
    dev = torch.device("cuda", torch.cuda.current_device())
    o = {"spins": torch.empty((R, N), dtype=torch.int8, device=dev),
         "best_step": torch.empty(R, dtype=torch.int32, device=dev),
         "x": torch.empty((R, N), dtype=torch.float32, device=dev),
         "y": torch.empty((R, N), dtype=torch.float32, device=dev)}
    for k in ("energy", "best_energy", "final_energy"):
        o[k] = torch.empty(R, dtype=torch.float64, device=dev)
    return o


def run(ctx, o, R, seed, steps=300, c0=None):
    c0 = 0.5 / np.sqrt(ctx.N) if c0 is None else c0
    ctx.run_ex(hsb.HSB_DSB, steps, R, 1.0, c0, 1.0, 0.01, seed=seed, want_state=True, out=o)
    torch.cuda.synchronize()
    return {k: o[k].cpu().numpy().copy() for k in KEYS}


def scramble(o):
    """Eager GPU work between launches: overwrite the outputs."""
    for t in o.values():
        t.fill_(7)
    torch.cuda.synchronize()


def assert_same(got, ref, what):
    for k in KEYS:
        assert np.array_equal(got[k], ref[k], equal_nan=True), f"{what}: {k}"


def eager_reference(J, R, seed, interval=50):
    with hsb.Context(J, precision="mixed", energy_interval=interval, graph=0) as ctx:
        o = outputs(R, J.shape[0])
        ref = run(ctx, o, R, seed)
        assert ctx.last_plan() == "fp4"
        assert ctx.get_option("graph_launches") == 0
    return ref


def test_graph_launches_equal_eager_run():
    N, R = 700, 96
    J = synth.sk_instance(N, 12)
    say("graph launches", N, R)
    ref = eager_reference(J, R, 5)
    # eager work on another context between the launches
    J2 = synth.sk_instance(300, 13)
    with hsb.Context(J, precision="mixed", energy_interval=50) as ctx, \
            hsb.Context(J2, precision="mixed", energy_interval=50, graph=0) as other:
        o = outputs(R, N)
        o2 = outputs(40, 300)
        for i in range(6):
            scramble(o)
            got = run(ctx, o, R, 5)
            assert_same(got, ref, f"call {i}")
            run(other, o2, 40, 9)
        # call 0 eager, call 1 captured and launched, calls 2-5 launched
        assert ctx.get_option("graph_launches") == 5


def test_graph_other_seed_and_dropped_by_other_runs():
    N, R = 500, 64
    J = synth.sk_instance(N, 14)
    say("graph seeds and drops", N, R)
    ref5 = eager_reference(J, R, 5)
    ref6 = eager_reference(J, R, 6)
    ref5_big = eager_reference(J, 2 * R, 5)
    with hsb.Context(J, precision="mixed", energy_interval=50) as ctx:
        o = outputs(R, N)
        for _ in range(3):
            assert_same(run(ctx, o, R, 5), ref5, "seed 5")
        assert ctx.get_option("graph_launches") == 2
        # the seed is read when the graph runs: another seed launches it too
        assert_same(run(ctx, o, R, 6), ref6, "seed 6")
        assert_same(run(ctx, o, R, 5), ref5, "seed 5 after 6")
        assert ctx.get_option("graph_launches") == 4
        # more replicas: the state is reallocated, the graph dropped
        ob = outputs(2 * R, N)
        assert_same(run(ctx, ob, 2 * R, 5), ref5_big, "2R")
        assert ctx.get_option("graph_launches") == 4
        # back to the first run: eager, then captured again on the new buffers
        for _ in range(3):
            scramble(o)
            assert_same(run(ctx, o, R, 5), ref5, "seed 5 again")
        assert ctx.get_option("graph_launches") == 6
        # a changed option changes the run: eager again
        ctx.set_option("return_best", 0)
        fin = run(ctx, o, R, 5)
        assert ctx.get_option("graph_launches") == 6
        assert np.array_equal(fin["x"], ref5["x"])  # same trajectory, other readout
        ctx.set_option("graph", 0)
        assert ctx.get_option("graph") == 0


def test_bsb_graph_launches_equal_eager_run():
    """bSB on the FP4 plan from a seeded state (INIT_AMP <= 1: no start-state
    check, so the run is graph-launched too)."""
    N, R = 300, 64
    J = synth.sk_instance(N, 15)
    c0 = 0.5 / np.sqrt(N)
    say("bsb graph launches", N, R)

    def bsb(ctx, o, seed):
        ctx.run_ex(hsb.HSB_BSB, 120, R, 1.0, c0, 1.0, 0.01, seed=seed, want_state=True, out=o)
        torch.cuda.synchronize()
        return {k: o[k].cpu().numpy().copy() for k in KEYS}

    with hsb.Context(J, precision="mixed", energy_interval=40, graph=0) as ctx:
        ref = bsb(ctx, outputs(R, N), 3)
        assert ctx.last_plan() == "fp4"
    with hsb.Context(J, precision="mixed", energy_interval=40) as ctx:
        o = outputs(R, N)
        for i in range(4):
            scramble(o)
            assert_same(bsb(ctx, o, 3), ref, f"bsb call {i}")
        assert ctx.get_option("graph_launches") == 3
