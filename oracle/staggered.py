"""Staggered lookup tables (Sec. III.B): the plain definitions of the entries.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

from ._clib import lib
from .combinatorics import cns_rank


def partrank(r: int, Mp: int, Np: int) -> int:
    """Eq. partrank: sum over the set bits c_1 < .. < c_Q of chunk r of
    C(M' + c_q, N' + q)."""
    return int(lib().orc_partrank(r, Mp, Np))


def partrank_reuse(r: int, Mp: int, Np: int) -> int:
    """Eq. reuse: the same entry as the combinadics rank of the pattern whose
    lowest N' bits are set and whose chunk r sits at offset M'."""
    return cns_rank((r << Mp) | ((1 << Np) - 1))


def chunk_widths(M: int, k: int) -> list:
    """Chunks of k bits from the least significant end; a final chunk holds the
    remaining M mod k bits when k does not divide M (the staggered loop simply
    runs out of bits)."""
    w, left = [], M
    while left > 0:
        w.append(min(k, left))
        left -= w[-1]
    return w


def staggered_rows(M: int, k: int, n_max: int):
    """Rows (chunk index c, M', N', width) needed to rank patterns of at most
    n_max particles: M' = c*k over the chunks, N' = 0..min(M', n_max)."""
    rows = []
    Mp = 0
    for c, w in enumerate(chunk_widths(M, k)):
        for Np in range(0, min(Mp, n_max) + 1):
            rows.append((c, Mp, Np, w))
        Mp += w
    return rows
