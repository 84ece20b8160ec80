"""Pins for oracle.combinatorics: paper examples, brute force, closed-form sizes."""
import json
import math
import os

import numpy as np
import pytest

from oracle import combinatorics as C

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_c34_example():
    g = GOLD["c34_ranks"]
    pats = [int(p, 2) for p in g["patterns"]]
    assert [C.cns_rank(p) for p in pats] == g["ranks"]
    s = C.sector_enumerate(4, C.constraints(4, 3))
    assert list(s) == pats
    assert list(C.bisect_rank(s, pats)) == g["ranks"]


def test_cns_example():
    g = GOLD["cns_example"]
    a = sum(1 << c for c in g["combination"])
    assert a == g["pattern"]
    assert C.cns_rank(a) == g["rank"]


def test_binomials_against_math_comb():
    for n in range(0, 65):
        for k in range(0, 66):
            assert C.binom(n, k) == (math.comb(n, k) if k <= n else 0)


@pytest.mark.parametrize("M", range(0, 13))
def test_bruteforce_all_sectors(M):
    for N in range(0, M + 1):
        cons = C.constraints(M, N)
        ref = C.sector_bruteforce(M, cons)
        s = C.sector_enumerate(M, cons)
        assert list(s) == ref
        assert len(ref) == math.comb(M, N)
        # rank = position, by both algorithms
        assert list(C.bisect_rank(s, s)) == list(range(len(ref)))
        assert list(C.cns_rank_batch(s)) == list(range(len(ref)))
        # unrank by greedy inversion = stored list
        assert [C.cns_unrank(i, N, M) for i in range(len(ref))] == ref


def test_bisect_rejects_non_members():
    s = C.sector_enumerate(10, C.constraints(10, 4))
    others = np.array([a for a in range(1 << 10) if bin(a).count("1") != 4] + [1 << 10, 2**40],
                      dtype=np.uint64)
    assert (C.bisect_rank(s, others) == -1).all()


def test_general_constraints_bruteforce():
    # extra window on the low 3 bits, with and without fixed N
    for cons in ([((1 << 9) - 1, 4, 4), (0b111, 2, 3)], [(0b111, 2, 3), (0b111000000, 0, 1)]):
        assert list(C.sector_enumerate(9, cons)) == C.sector_bruteforce(9, cons)


def test_spin_product_size_and_order():
    for L, nu, nd in [(3, 1, 2), (4, 2, 2), (4, 1, 3), (5, 2, 1)]:
        s = C.sector_enumerate(2 * L, C.spin_constraints(L, nu, nd))
        assert s.size == math.comb(L, nu) * math.comb(L, nd)
        assert (np.diff(s.astype(np.int64)) > 0).all()


def test_ras_sector_size_closed_form():
    # popcount 16 of 32 with >= 6 set among bits 0..7 (sizes only; M = 32 walk takes seconds)
    want = sum(math.comb(8, a) * math.comb(24, 16 - a) for a in range(6, 9))
    assert want == 66110671
    # reduced instance checked exhaustively: M = 16, N = 8, >= 3 of bits 0..3
    cons = C.constraints(16, 8, [(0xF, 3, 4)])
    s = C.sector_enumerate(16, cons)
    assert s.size == sum(math.comb(4, a) * math.comb(12, 8 - a) for a in (3, 4))
    assert list(s) == C.sector_bruteforce(16, cons)


def test_binomial_table_size_m64():
    g = GOLD["binomial_table_bytes_M64"]
    # table C(c, k) for 0 <= c < 64, 1 <= k <= 64 of 64-bit numbers
    assert 64 * 64 * 8 == g["bytes"]
    assert max(C.binom(c, k) for c in range(64) for k in range(1, 65)) < 2 ** 64
