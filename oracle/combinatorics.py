"""Sectors, combinadics and bisection: the plain definitions of rank and unrank.

Test infrastructure only (see the package docstring).  Follows Sec. II-III of
Wallerberger & Held, arXiv:2203.04158: a state is an M-bit occupation pattern
(bit i = orbital i), a sector is the ordered set of patterns with given
quantum numbers, rank = position in that ordered set, unrank = its inverse.
"""
from __future__ import annotations

import numpy as np

from ._clib import lib, ptr


def binom(n: int, k: int) -> int:
    """C(n, k) with C(n, k) = 0 for k > n (convention under Eq. cns)."""
    return int(lib().orc_binom(n, k))


def cns_rank(alpha: int) -> int:
    """Eq. cns / Eq. rank: sum of C(c_k, k) over the occupied positions c_1 < ... < c_N."""
    return int(lib().orc_cns_rank(alpha))


def cns_rank_batch(q) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.uint64)
    out = np.empty_like(q)
    lib().orc_cns_rank_batch(ptr(q), q.size, ptr(out))
    return out


def cns_unrank(idx: int, N: int, M: int) -> int:
    """Eq. unrank: greedy inversion of Eq. cns."""
    return int(lib().orc_cns_unrank(idx, N, M))


def constraints(M: int, N: int | None = None, extra=()):
    """Constraint list [(mask, lo, hi)]: optional total particle number N on all
    M bits, plus any extra (mask, lo, hi) popcount windows."""
    cons = []
    if N is not None:
        cons.append(((1 << M) - 1, N, N))
    cons.extend(extra)
    return cons


def spin_constraints(L: int, n_up: int, n_dn: int):
    """(N_up, N_dn) sector of 2L spin-orbitals, spin-down in the low L bits
    (assumption stated with Eq. rankupdown)."""
    lo_mask = (1 << L) - 1
    return [(((1 << (2 * L)) - 1), n_up + n_dn, n_up + n_dn),
            (lo_mask, n_dn, n_dn), (lo_mask << L, n_up, n_up)]


def sector_enumerate(M: int, cons) -> np.ndarray:
    """All M-bit patterns satisfying every (mask, lo, hi) popcount window, in
    ascending numeric order (= lexicographic order of Sec. III)."""
    nc = len(cons)
    mask = np.array([c[0] for c in cons] or [0], dtype=np.uint64)
    lo = np.array([c[1] for c in cons] or [0], dtype=np.int32)
    hi = np.array([c[2] for c in cons] or [0], dtype=np.int32)
    full = (1 << M) - 1
    fixed = -1
    for c in cons:
        if c[0] == full and c[1] == c[2]:
            fixed = c[1]
    L = lib()
    n = L.orc_sector_enumerate(M, nc, ptr(mask), ptr(lo), ptr(hi), fixed, None, 0)
    if n < 0:
        raise ValueError("sector too large for the oracle enumerator")
    out = np.empty(n, dtype=np.uint64)
    L.orc_sector_enumerate(M, nc, ptr(mask), ptr(lo), ptr(hi), fixed, ptr(out), n)
    return out


def sector_bruteforce(M: int, cons) -> list:
    """Pure-Python filter over all 2^M patterns (tiny M only)."""
    return [a for a in range(1 << M)
            if all(lo <= bin(a & m).count("1") <= hi for (m, lo, hi) in cons)]


def bisect_rank(states, q) -> np.ndarray:
    """Bisection in the sorted list (the established method); -1 = not in sector."""
    states = np.ascontiguousarray(states, dtype=np.uint64)
    q = np.ascontiguousarray(q, dtype=np.uint64)
    out = np.empty(q.size, dtype=np.int64)
    lib().orc_bisect_rank_batch(ptr(states), states.size, ptr(q), q.size, ptr(out))
    return out


def unrank(states, idx) -> np.ndarray:
    """Unrank by the stored list (Sec. II): unrank(i) = states[i]."""
    return np.asarray(states)[np.asarray(idx)]


def rank_batch_threads(states, q, method: str, threads: int) -> np.ndarray:
    """bisect_rank ('bisect') or cns_rank_batch ('cns') over `threads` OpenMP
    threads (timing leg only; same results as the single-thread functions)."""
    states = np.ascontiguousarray(states, dtype=np.uint64)
    q = np.ascontiguousarray(q, dtype=np.uint64)
    out = np.empty(q.size, dtype=np.int64)
    lib().orc_rank_batch_mt(ptr(states), states.size, ptr(q), q.size, ptr(out),
                            0 if method == "bisect" else 1, threads)
    return out
