"""Seeded synthetic inputs: Ising instances and their sizes.

This module holds no arithmetic of the method itself. It only produces the
coupling matrices J (and, for batched workloads, the instance sizes) that both
the GPU path and the CPU oracle consume, so that both sides start from the
same problem.

The paper benchmarks on K2000 and on 100 instances of a 700-spin problem
(Results, "Performance for a 2000-spin Ising problem" and "... 100 instances
of a 700-spin Ising problem"); neither set is available here. The generators
below produce instances of the same shape and distribution: all-to-all,
symmetric, zero diagonal, J_ij = +1 or -1 with equal probability (the SK
model, Results, paragraph after eq. (11)), plus a Gaussian variant
J_ij ~ N(0, 1)/sqrt(N).

Random numbers come from a counter-based generator built on the output mixer
of SplitMix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014):

    mix(z)  = z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
              z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31
    key(seed, stream, a, b) = mix(mix(mix(seed + G*(stream+1)) + G*(a+1)) + G*(b+1))

with G = 0x9E3779B97F4A7C15 and all arithmetic modulo 2**64.  Streams:
0 = initial x, 1 = initial y (drawn inside the library and the oracle, each
with its own implementation), 2 = SK coupling signs, 3 = batched instance
sizes, 4 and 5 = Gaussian couplings (Box-Muller uniforms).
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

STREAM_X, STREAM_Y, STREAM_SK, STREAM_SIZES, STREAM_GAUSS_U1, STREAM_GAUSS_U2 = range(6)


def _mix(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def key(seed: int, stream: int, a, b) -> np.ndarray:
    """Counter-based 64-bit hash of (seed, stream, a, b); a and b broadcast."""
    with np.errstate(over="ignore"):
        s = np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
        h = _mix(s + GOLDEN * np.uint64(stream + 1))
        a = np.asarray(a, dtype=np.uint64)
        b = np.asarray(b, dtype=np.uint64)
        h = _mix(h + GOLDEN * (a + np.uint64(1)))
        h = _mix(h + GOLDEN * (b + np.uint64(1)))
    return h


def uniform_open(seed: int, stream: int, a, b) -> np.ndarray:
    """float32 values in the open interval (-1, 1), never 0, exactly representable.

    m = top 24 bits of the hash; v = (2m + 1 - 2**24) * 2**-24.
    """
    m = (key(seed, stream, a, b) >> np.uint64(40)).astype(np.int64)
    return ((2 * m + 1 - (1 << 24)).astype(np.float64) * 2.0 ** -24).astype(np.float32)


def sk_instance(N: int, seed: int) -> np.ndarray:
    """SK instance: float32 N x N, symmetric, zero diagonal, J_ij = +-1 equiprobable."""
    if N < 1:
        raise ValueError("N must be >= 1")
    i, j = np.triu_indices(N, k=1)
    bits = key(seed, STREAM_SK, i, j) >> np.uint64(63)
    vals = np.where(bits == 1, -1.0, 1.0).astype(np.float32)
    J = np.zeros((N, N), dtype=np.float32)
    J[i, j] = vals
    J[j, i] = vals
    return J


def gaussian_instance(N: int, seed: int) -> np.ndarray:
    """Gaussian SK instance: J_ij = z / sqrt(N), z ~ N(0,1) by Box-Muller in FP64, stored FP32."""
    if N < 1:
        raise ValueError("N must be >= 1")
    i, j = np.triu_indices(N, k=1)
    k1 = key(seed, STREAM_GAUSS_U1, i, j) >> np.uint64(11)
    k2 = key(seed, STREAM_GAUSS_U2, i, j) >> np.uint64(11)
    u1 = (k1.astype(np.float64) + 0.5) * 2.0 ** -53
    u2 = (k2.astype(np.float64) + 0.5) * 2.0 ** -53
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    vals = (z / np.sqrt(N)).astype(np.float32)
    J = np.zeros((N, N), dtype=np.float32)
    J[i, j] = vals
    J[j, i] = vals
    return J


def uneven_sizes(count: int, seed: int, lo: int = 100, hi: int = 2000) -> np.ndarray:
    """Instance sizes uniform on [lo, hi] (inclusive) for batched workloads."""
    t = np.arange(count, dtype=np.uint64)
    h = key(seed, STREAM_SIZES, t, 0)
    return (lo + (h % np.uint64(hi - lo + 1)).astype(np.int64)).astype(np.int64)


def ferromagnet(N: int, scale: float = 1.0) -> np.ndarray:
    """All couplings equal (J_ij = scale for i != j): ground states are the two aligned states."""
    J = np.full((N, N), scale, dtype=np.float32)
    np.fill_diagonal(J, 0.0)
    return J
