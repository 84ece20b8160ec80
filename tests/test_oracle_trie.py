"""Pins for oracle.trie: the worked example and the printed overhead factors."""
import json
import os

import numpy as np
import pytest

from oracle import combinatorics as C
from oracle import trie as T

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_worked_example():
    g = GOLD["trie_example"]
    s = C.sector_enumerate(g["M"], C.constraints(g["M"], g["N"]))
    w = T.chunk_widths(g["M"], g["R"])
    t = T.build(s, w, tail_pad=False)
    for k, v in g["slots"].items():
        assert t[int(k)] == v
    assert T.lookup(t, int(g["query"], 2), w) == g["rank"]
    assert round(len(t) / s.size, 6) == g["f_approx"]
    assert T.packed_size(s, w) == len(t)


@pytest.mark.parametrize("M,N,R", [(6, 2, 2), (8, 3, 3), (10, 5, 4), (12, 4, 5), (9, 4, 2), (7, 3, 7)])
def test_lookup_all_members(M, N, R):
    s = C.sector_enumerate(M, C.constraints(M, N))
    for short in ("last", "first"):
        w = T.chunk_widths(M, R, short)
        t = T.build(s, w)
        assert [T.lookup(t, int(a), w) for a in s] == list(range(s.size))
        # safe lookup: every M-bit pattern stays in bounds; membership via the list
        for a in range(1 << M):
            i = T.lookup(t, a, w)
            member = i < s.size and int(s[i]) == a
            assert member == (bin(a).count("1") == N)


def test_irregular_sector_lookup():
    cons = C.constraints(10, 5, [(0b111, 2, 3)])
    s = C.sector_enumerate(10, cons)
    w = T.chunk_widths(10, 3)
    t = T.build(s, w)
    assert [T.lookup(t, int(a), w) for a in s] == list(range(s.size))


@pytest.mark.slow
def test_overhead_factors_m28():
    # The printed factors come out when the first-dispatched chunk is the short one.
    g = GOLD["trie_overhead"]
    for key, N in (("N14", 14), ("N5", 5)):
        s = C.sector_enumerate(28, C.constraints(28, N))
        for R, want in g[key].items():
            f = T.packed_size(s, T.chunk_widths(28, int(R), "first")) / s.size
            assert round(f, 2) == want


def test_overhead_factor_n5_fast():
    g = GOLD["trie_overhead"]
    s = C.sector_enumerate(28, C.constraints(28, 5))
    for R, want in g["N5"].items():
        f = T.packed_size(s, T.chunk_widths(28, int(R), "first")) / s.size
        assert round(f, 2) == want
