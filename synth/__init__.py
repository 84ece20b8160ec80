"""Seeded synthetic inputs shared by the oracle-side tests and the HIP-side tests/bench.

This module holds random-number generation and input recipes only; it contains
none of the ranking or Hamiltonian arithmetic.  Every stream is SplitMix64
(S. Vigna's published 64-bit mixer), evaluated in closed form for index k as
mix(seed + (k + 1) * 0x9E3779B97F4A7C15), so any element can be regenerated
independently and both sides see byte-identical inputs.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Elements start..start+n-1 of the SplitMix64 stream for `seed` (uint64)."""
    k = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform01(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of each SplitMix64 draw."""
    return (splitmix64(seed, n, start) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_indices(seed: int, n: int, bound: int) -> np.ndarray:
    """n indices in [0, bound) as draw mod bound (bias below bound / 2^64)."""
    return (splitmix64(seed, n) % np.uint64(bound)).astype(np.int64)


def start_vector(seed: int, n: int) -> np.ndarray:
    """Lanczos start vector: entries uniform in [-1, 1), scaled to unit norm (fp64)."""
    v = 2.0 * uniform01(seed, n) - 1.0
    return v / np.sqrt(np.dot(v, v))


def random_subset_patterns(seed: int, n: int, M: int, N: int) -> np.ndarray:
    """n patterns with exactly N of M bits set, each uniform over all such patterns.

    Each pattern picks N distinct positions by a partial Fisher-Yates shuffle
    driven by the stream (positions drawn as value mod remaining)."""
    raw = splitmix64(seed, n * N).reshape(n, N) if N > 0 else np.zeros((n, 0), np.uint64)
    out = np.zeros(n, dtype=np.uint64)
    pos = np.tile(np.arange(M, dtype=np.int64), (n, 1))
    rows = np.arange(n)
    for j in range(N):
        pick = j + (raw[:, j] % np.uint64(M - j)).astype(np.int64)
        a = pos[rows, j].copy()
        pos[rows, j] = pos[rows, pick]
        pos[rows, pick] = a
        out |= np.uint64(1) << pos[rows, j].astype(np.uint64)
    return out


def anderson_parameters(seed: int, n_bath: int):
    """Bath levels eps_l uniform in [-2, 2] and hybridisations V_l uniform in
    [0.2, 0.8]: eps_1..eps_nb from the first n_bath draws, V_1..V_nb from the next."""
    u = uniform01(seed, 2 * n_bath)
    eps = -2.0 + 4.0 * u[:n_bath]
    V = 0.2 + 0.6 * u[n_bath:]
    return eps, V


def shuffle_positions(seed: int, n: int) -> np.ndarray:
    """A seeded permutation of 0..n-1 (argsort of the stream; ties impossible in practice)."""
    return np.argsort(splitmix64(seed, n), kind="stable")
