"""Pins for the oracle's definitions: generator, eq. (1), eqs. (13)-(14), brute force, eqs. (4)-(5).

Each test fixes the oracle against something other than its own code: published
generator outputs, hand-worked values, closed forms, invariances of eq. (1), an
independent numpy formulation, or exhaustive search.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth


def _load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as fh:
        return json.load(fh)


# ------------------------------------------------------------------ generator

def test_splitmix64_published_outputs(golden_dir):
    g = _load(golden_dir, "splitmix64.json")
    for stream, hexval in enumerate(g["seed0_outputs_hex"]):
        # first stage of key(seed=0, stream, .) is mix(G*(stream+1))
        expect = int(hexval, 16)
        G = 0x9E3779B97F4A7C15
        M = (1 << 64) - 1
        z = (G * (stream + 1)) & M
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        z = z ^ (z >> 31)
        assert z == expect  # this file's transcription of the published mixer
    # full chain agrees between the oracle (C) and the input module (numpy),
    # two independent implementations of the same published definition
    for (seed, stream, a, b) in [(0, 0, 0, 0), (1, 1, 5, 7), (2**63 + 12345, 2, 1999, 3),
                                 (42, 3, 0, 2**20)]:
        assert oracle.key(seed, stream, a, b) == int(synth.key(seed, stream, a, b)[0])


def test_first_stage_is_splitmix_output(golden_dir):
    g = _load(golden_dir, "splitmix64.json")
    first = int(g["seed0_outputs_hex"][0], 16)
    # key(0, 0, a, b) = mix(mix(first + G(a+1)) + G(b+1)); numpy side built from `first`
    G = 0x9E3779B97F4A7C15
    M = (1 << 64) - 1

    def mix(z):
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)

    for a, b in [(0, 0), (3, 9), (1023, 1999)]:
        assert oracle.key(0, 0, a, b) == mix((mix((first + G * (a + 1)) & M) + G * (b + 1)) & M)


def test_uniform_open_interval_properties():
    N, R = 4096, 16
    x0, y0 = oracle.init_state(7, R, N, amp=1.0)
    for v in (x0, y0):
        assert np.all(np.abs(v) < 1.0)
        assert np.all(v != 0.0)
        # values are odd multiples of 2^-24
        m = v.astype(np.float64) * 2.0 ** 24
        assert np.all(m == np.round(m)) and np.all(np.mod(np.round(m), 2) == 1)
        # moments of U(-1, 1): mean 0 (sd 1/sqrt(3n)), variance 1/3
        n = v.size
        assert abs(v.mean()) < 5.0 / np.sqrt(3 * n)
        assert abs(v.var() - 1.0 / 3.0) < 5.0 * np.sqrt(4.0 / 45.0 / n)
    # x and y use different streams
    assert not np.array_equal(x0, y0)


def test_init_amplitude_is_one_rounding():
    x1, _ = oracle.init_state(3, 2, 64, amp=1.0)
    x01, _ = oracle.init_state(3, 2, 64, amp=0.1)
    assert np.array_equal(x01, (np.float32(0.1) * x1).astype(np.float32))
    # replica block offset: replica r depends only on (seed, r)
    xa, ya = oracle.init_state(3, 5, 64, amp=0.1)
    xb, yb = oracle.init_state(3, 2, 64, amp=0.1, r0=3)
    assert np.array_equal(xa[3:], xb) and np.array_equal(ya[3:], yb)


# ------------------------------------------------------------------ eq. (1), (13), (14)

def test_energy_and_cut_hand_cases(golden_dir):
    g = _load(golden_dir, "energy_cases.json")
    for c in g["cases"]:
        J = np.array(c["J"], dtype=np.float64)
        s = np.array(c["s"], dtype=np.int8)
        assert oracle.energy(J, s) == c["E"], c["name"]
        assert oracle.cut(J, s) == c["C"], c["name"]
    for c in g["ground_states"]:
        e, s, n = oracle.brute_force(np.array(c["J"], dtype=np.float64))
        assert e == c["E_min"] and n == c["n_min"]


@pytest.mark.parametrize("N,seed", [(5, 1), (16, 2), (40, 3)])
def test_cut_identity_eq14(N, seed):
    J = synth.sk_instance(N, seed)
    rng = np.random.default_rng(seed)
    for _ in range(5):
        s = rng.choice([-1, 1], size=N).astype(np.int8)
        E = oracle.energy(J, s)
        C = oracle.cut(J, s)
        assert C == -0.5 * E - 0.25 * float(J.astype(np.float64).sum())  # exact: integers


@pytest.mark.parametrize("N,seed", [(7, 4), (33, 5)])
def test_energy_invariances(N, seed):
    for J in (synth.sk_instance(N, seed), synth.gaussian_instance(N, seed)):
        rng = np.random.default_rng(seed)
        s = rng.choice([-1, 1], size=N).astype(np.int8)
        d = rng.choice([-1, 1], size=N).astype(np.int8)
        E = oracle.energy(J, s)
        assert oracle.energy(J, -s) == E  # global flip
        Jg = (d[:, None] * J.astype(np.float64) * d[None, :])
        assert oracle.energy(Jg, d * s) == pytest.approx(E, rel=1e-14, abs=1e-12)  # gauge
        # independent formulation: -1/2 s^T J s with a library product
        Sd = s.astype(np.float64)
        assert oracle.energy(J, s) == pytest.approx(-0.5 * Sd @ J.astype(np.float64) @ Sd,
                                                    rel=1e-13, abs=1e-12)


# ------------------------------------------------------------------ brute force

def _numpy_exhaustive(J):
    N = J.shape[0]
    m = np.arange(1 << N)[:, None]
    S = np.where((m >> np.arange(N)[None, :]) & 1, -1.0, 1.0)
    E = -0.5 * np.einsum("ki,ij,kj->k", S, J.astype(np.float64), S)
    return E.min(), int(np.sum(E == E.min()))


@pytest.mark.parametrize("N,seed", [(6, 1), (10, 2), (12, 3)])
def test_brute_force_matches_independent_enumeration(N, seed):
    J = synth.sk_instance(N, seed)
    e, s, n = oracle.brute_force(J)
    e2, n2 = _numpy_exhaustive(J)
    assert e == e2 and n == n2
    assert oracle.energy(J, s) == e
    assert n % 2 == 0  # minimisers come in global-flip pairs


@pytest.mark.parametrize("N", [2, 5, 9])
def test_brute_force_closed_forms(N):
    # ferromagnet: two aligned ground states with E = -N(N-1)/2
    e, s, n = oracle.brute_force(synth.ferromagnet(N))
    assert e == -N * (N - 1) / 2 and n == 2 and abs(int(s.sum())) == N
    # Mattis model J_ij = xi_i xi_j: ground states +-xi with the same energy
    xi = np.where(np.arange(N) % 3 == 1, -1, 1).astype(np.int8)
    J = np.outer(xi, xi).astype(np.float64)
    np.fill_diagonal(J, 0.0)
    e, s, n = oracle.brute_force(J)
    assert e == -N * (N - 1) / 2 and n == 2
    assert np.array_equal(s, xi) or np.array_equal(s, -xi)


# ------------------------------------------------------------------ eqs. (4), (5)

@pytest.mark.parametrize("N,seed", [(17, 1), (200, 2)])
def test_field_bsb_is_matrix_product(N, seed):
    for J in (synth.sk_instance(N, seed), synth.gaussian_instance(N, seed)):
        x = np.random.default_rng(seed).uniform(-1, 1, N)
        f = oracle.field(J, x, oracle.BSB)
        ref = J.astype(np.float64) @ x
        assert np.allclose(f, ref, rtol=1e-13, atol=1e-13 * np.abs(J).sum(1).max())


@pytest.mark.parametrize("N,seed", [(17, 1), (200, 2)])
def test_field_dsb_exact_integers(N, seed):
    J = synth.sk_instance(N, seed)
    x = np.random.default_rng(seed).uniform(-1, 1, N)
    f = oracle.field(J, x, oracle.DSB)
    s = np.where(x >= 0, 1, -1).astype(np.int64)
    assert np.array_equal(f, (J.astype(np.int64) @ s).astype(np.float64))


def test_sign_convention_zero_is_plus():
    J = np.array([[0, 1, 1], [1, 0, 1], [1, 1, 0]], dtype=np.float64)
    x = np.array([0.0, -0.0, -0.5])
    f = oracle.field(J, x, oracle.DSB)
    # sgn(0) = sgn(-0) = +1, sgn(-0.5) = -1
    assert np.array_equal(f, [0.0, 0.0, 2.0])


def test_sk_instance_shape_and_distribution():
    J = synth.sk_instance(300, 9)
    assert np.array_equal(J, J.T) and np.all(np.diag(J) == 0)
    off = J[~np.eye(300, dtype=bool)]
    assert set(np.unique(off)) == {-1.0, 1.0}
    frac = (off > 0).mean()
    assert abs(frac - 0.5) < 5 * 0.5 / np.sqrt(off.size / 2)
    G = synth.gaussian_instance(300, 9)
    assert np.array_equal(G, G.T) and np.all(np.diag(G) == 0)
    goff = G[np.triu_indices(300, 1)].astype(np.float64) * np.sqrt(300)
    assert abs(goff.mean()) < 5 / np.sqrt(goff.size) and abs(goff.std() - 1) < 0.02
    sizes = synth.uneven_sizes(256, 4)
    assert sizes.min() >= 100 and sizes.max() <= 2000
