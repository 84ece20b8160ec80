"""Sectors adopted from a caller's list (mbr_sector_from_list): the list is
checked on the device (ENOTSORTED, EDUP, bits at or above M), and a trie built
on an adopted irregular sector ranks it bit-exactly against the oracle's
bisection (Sec. IV: irregular sets are fed to the trie builder in order)."""
import numpy as np
import pytest

from oracle import combinatorics as OC
import synth
from tests._util import dev_u32, dev_u64, host_u32, host_u64, host_rank, say

pytestmark = pytest.mark.gpu

mbr = pytest.importorskip("paper_2203_04158_amd")


def _momentum_list(L, nu, nd, K):
    """The oracle's total-momentum sector of a ring: spin sector (nu, nd) of 2L
    orbitals whose momenta (orbital i and L+i carry momentum i) add up to K mod L."""
    st = OC.sector_enumerate(2 * L, OC.spin_constraints(L, nu, nd))
    w = np.array([i % L for i in range(2 * L)], dtype=np.int64)
    bits = (st[:, None] >> np.arange(2 * L, dtype=np.uint64)) & np.uint64(1)
    keep = (bits.astype(np.int64) @ w) % L == K
    return st[keep]


@pytest.mark.parametrize("k", [4, 8])
def test_from_list_trie_ranks_irregular_sector(k):
    L, nu, nd, K = 8, 4, 3, 2
    st = _momentum_list(L, nu, nd, K)
    say("from_list momentum sector", L, nu, nd, K, st.size, "k", k)
    s = mbr.sector_from_list(2 * L, dev_u32(st))
    assert s.size == st.size
    assert np.array_equal(host_u32(s.states()), st)
    r = mbr.build_trie(s, k)
    full = OC.sector_enumerate(2 * L, OC.spin_constraints(L, nu, nd))
    rng = synth.uniform_indices(91, 20000, full.size)
    q = np.concatenate([st, full[rng], synth.splitmix64(92, 5000) & np.uint64((1 << (2 * L + 2)) - 1)])
    got = host_rank(mbr.rank_batch(r, dev_u32(q)))
    assert np.array_equal(got, OC.bisect_rank(st, q))


def test_from_list_matches_modular_build():
    L, nu, nd, K = 10, 5, 5, 0
    st = _momentum_list(L, nu, nd, K)
    a = mbr.sector_from_list(2 * L, dev_u32(st))
    b = mbr.sector_build_mod(2 * L, OC.spin_constraints(L, nu, nd), [i % L for i in range(2 * L)], L, K)
    assert a.size == b.size == st.size
    assert np.array_equal(host_u32(a.states()), host_u32(b.states()))


def test_from_list_u64_and_empty():
    st = OC.sector_enumerate(40, OC.constraints(40, 2))
    s = mbr.sector_from_list(40, dev_u64(st), width_bits=64)
    assert s.size == st.size
    assert np.array_equal(host_u64(s.states()), st)
    r = mbr.build_trie(s, 8)
    q = np.concatenate([st[::7], np.array([0, 3 << 38, (1 << 40) - 1], dtype=np.uint64)])
    got = host_rank(mbr.rank_batch(r, dev_u64(q)))
    assert np.array_equal(got, OC.bisect_rank(st, q))
    import torch
    e = mbr.sector_from_list(12, torch.empty(0, dtype=torch.int32, device="cuda"))
    assert e.size == 0


def _expect(status, M, lst, width=32, text=None):
    with pytest.raises(mbr.MbrError) as ei:
        mbr.sector_from_list(M, dev_u32(lst) if width == 32 else dev_u64(lst), width_bits=width)
    assert ei.value.status == status
    if text:
        assert text in str(ei.value), str(ei.value)


def test_from_list_rejects_bad_lists():
    st = OC.sector_enumerate(16, OC.constraints(16, 5)).copy()   # 4368 states
    uns = st.copy()
    uns[3000], uns[3001] = uns[3001], uns[3000]
    _expect(-4, 16, uns, text="entry 3001 is smaller than entry 3000")
    dup = st.copy()
    dup[1234] = dup[1233]
    _expect(-5, 16, dup, text="entry 1234 repeats entry 1233")
    # both faults: the first position decides
    both = st.copy()
    both[100] = both[99]
    both[4000], both[4001] = both[4001], both[4000]
    _expect(-5, 16, both, text="entry 100")
    both = st.copy()
    both[4000] = both[3999]
    both[10], both[11] = both[11], both[10]
    _expect(-4, 16, both, text="entry 11")
    wide = st.copy()
    wide[-1] = 1 << 16          # still ascending, but bit 16 is outside M = 16
    _expect(-1, 16, wide, text="bits at or above M")
    big = OC.sector_enumerate(40, OC.constraints(40, 2))
    bad = big.copy()
    bad[500] = bad[501]
    _expect(-5, 40, bad, width=64, text="entry 501 repeats entry 500")
    # a strictly ascending list of arbitrary patterns is accepted
    ok = np.unique(synth.splitmix64(93, 100000) & np.uint64((1 << 24) - 1))
    assert mbr.sector_from_list(24, dev_u32(ok)).size == ok.size
