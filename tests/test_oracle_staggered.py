"""Pins for oracle.staggered: Eq. partrank against Eq. reuse and against Eq. cns."""
import numpy as np
import pytest

from oracle import combinatorics as C
from oracle import staggered as S
from synth import splitmix64


@pytest.mark.parametrize("R", [1, 2, 3, 4, 8])
def test_partrank_equals_reuse(R):
    for Mp in range(0, 20, 3):
        for Np in range(0, Mp + 1):
            for r in range(1 << R):
                assert S.partrank(r, Mp, Np) == S.partrank_reuse(r, Mp, Np)


@pytest.mark.parametrize("M,k", [(24, 8), (28, 7), (28, 14), (32, 8), (14, 7), (14, 14),
                                 (13, 5), (40, 11), (64, 8)])
def test_chunked_sum_equals_cns(M, k):
    # Summing Eq. partrank over the chunks (M' and N' advanced as in the
    # staggered loop) reproduces Eq. cns for arbitrary patterns.
    q = splitmix64(7 + M + k, 2000)
    if M < 64:
        q = q & np.uint64((1 << M) - 1)
    ref = C.cns_rank_batch(q)
    w = S.chunk_widths(M, k)
    for a, want in zip(q.tolist(), ref.tolist()):
        tot, Mp, Np, rest = 0, 0, 0, a
        for wc in w:
            r = rest & ((1 << wc) - 1)
            tot += S.partrank(r, Mp, Np)
            Mp += wc
            Np += bin(r).count("1")
            rest >>= wc
        assert tot == want


def test_rows_direct_count():
    # M = 24, k = 8, N <= 12: M' in {0, 8, 16} -> 1 + 9 + 13 rows
    assert len(S.staggered_rows(24, 8, 12)) == 23
    # universal table at M = 64, k = 8: sum over M' = 0, 8, .., 56 of (M' + 1) rows
    assert len(S.staggered_rows(64, 8, 64)) == sum(m + 1 for m in range(0, 64, 8)) == 232
