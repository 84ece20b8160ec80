"""GPU parity of trie ranking (bit-exact) and its memory footprint."""
import math

import numpy as np
import pytest

from oracle import combinatorics as OC
from oracle import trie as OT
import synth
from tests._util import dev_u32, dev_u64, host_rank, say

pytestmark = pytest.mark.gpu
mbr = pytest.importorskip("paper_2203_04158_amd")


def _expected_entries(states, M, k):
    """Entries of the GPU layout: the paper's packed count (chunks of k from the
    least significant end, short chunk last) with the root widened to all 2^w0
    slots, plus 2^w - 1 leading and 2^w trailing zeros on every other level."""
    w = OT.chunk_widths(M, k, "last")
    packed = OT.packed_size(states, w)
    c0 = np.asarray(states, dtype=np.uint64) & np.uint64((1 << w[0]) - 1)
    root_span = int(c0.max()) - int(c0.min()) + 1
    return packed - root_span + (1 << w[0]) + sum(2 * (1 << wl) - 1 for wl in w[1:])


def _check(M, cons, k, width=32, n_noise=20000, seed=1):
    st = OC.sector_enumerate(M, cons)
    s = mbr.sector_build(M, cons, width_bits=width)
    assert s.size == st.size
    r = mbr.build_trie(s, k)
    info = r.info()
    assert info.levels == -(-M // k)
    ent, lds_lv = mbr.trie_level_entries(r)
    assert len(ent) == info.levels and 4 * sum(ent) == info.bytes and 0 <= lds_lv <= info.levels
    assert mbr.trie_bytes(r) == info.bytes
    assert ent[0] == 1 << OT.chunk_widths(M, k, "last")[0]  # the root is a full node
    if M - OT.chunk_widths(M, k, "last")[-1] <= 26:  # range of the oracle's size counter
        assert info.bytes == 4 * _expected_entries(st, M, k)
    dev = dev_u32 if width == 32 else dev_u64
    got = host_rank(mbr.rank_batch(r, dev(st)))
    assert np.array_equal(got, np.arange(st.size))
    lim = (1 << M) - 1 if M < 64 else (1 << 64) - 1
    noise = synth.splitmix64(seed + M * 97 + k, n_noise) & np.uint64(lim)
    over = (st[: min(1000, st.size)] | np.uint64(1 << M)) if M < width else np.zeros(0, np.uint64)
    q = np.concatenate([noise, over, st[::max(1, st.size // 500)]])
    got = host_rank(mbr.rank_batch(r, dev(q)))
    assert np.array_equal(got, OC.bisect_rank(st, q))
    return r


def test_worked_example_sector():
    _check(6, OC.constraints(6, 2), 2)


@pytest.mark.parametrize("M,N,k", [(12, 6, 1), (12, 6, 2), (13, 5, 3), (16, 8, 4), (16, 8, 5),
                                   (20, 10, 8), (24, 12, 8), (16, 3, 16), (17, 8, 16), (9, 0, 4),
                                   (9, 9, 4)])
def test_particle_number_sectors(M, N, k):
    say("trie", M, N, k)
    _check(M, OC.constraints(M, N), k)


@pytest.mark.parametrize("k", [3, 4, 8])
def test_irregular_sectors(k):
    _check(20, OC.constraints(20, 10, [(0xFF, 6, 8)]), k)           # RAS-like
    _check(18, [(0x3FFFF, 7, 9), (0x5555, 2, 5)], k)                 # mixed N
    _check(24, OC.spin_constraints(12, 6, 5), k)                     # spin product


def test_u64_sector():
    _check(40, OC.constraints(40, 3, [(0xF, 1, 2)]), 8, width=64)


@pytest.mark.parametrize("k", [4, 8])
def test_ras_m32_full_size(k):
    """M = 32, N = 16 with at least 6 of orbitals 0-7 occupied (66,110,671
    states); 2^24 queries, 90% members drawn uniformly by index and 10%
    popcount-16 patterns with at most 5 of orbitals 0-7 occupied."""
    M = 32
    cons = OC.constraints(M, 16, [(0xFF, 6, 8)])
    st = OC.sector_enumerate(M, cons)
    assert st.size == 66110671
    s = mbr.sector_build(M, cons)
    r = mbr.build_trie(s, k)
    say("ras trie k", k, "bytes", r.info().bytes, "f", r.info().bytes / 4 / st.size)
    nq = 1 << 24
    nm = nq // 10
    idx = synth.uniform_indices(3, nq - nm, st.size)
    pool = synth.random_subset_patterns(33, 3 * nm, 32, 16)
    low = np.array([bin(int(v) & 0xFF).count("1") for v in pool])
    non = pool[low <= 5][:nm]
    assert non.size == nm
    q = np.concatenate([st[idx], non])
    perm = synth.shuffle_positions(34, q.size)
    q = q[perm]
    want = np.concatenate([idx, np.full(nm, -1)])[perm]
    got = host_rank(mbr.rank_batch(r, dev_u32(q)))
    assert np.array_equal(got, want)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("N", [14, 5])
def test_m28_k12(N):
    """R = 12 at M = 28, the largest chunk width of the paper's sweep (Sec.
    V.A): chunks of 12, 12 and 4 bits; half filling (40,116,600 states) and
    N = 5 (98,280), where the trie is mostly padding.  Every member, seeded
    arbitrary 28-bit and 29-bit patterns, sizes against the packed count."""
    r = _check(28, OC.constraints(28, N), 12, n_noise=1 << 20, seed=N)
    say("M=28 N", N, "k=12 bytes", r.info().bytes)


def test_trie_rejects_bad_args():
    s = mbr.sector_build(10, OC.constraints(10, 5))
    with pytest.raises(mbr.MbrError):
        mbr.build_trie(s, 0)
    with pytest.raises(mbr.MbrError):
        mbr.build_trie(s, 17)


def _bt_check(M, cons, k, width=32, n_noise=20000, seed=1):
    """Bitmap trie: every member ranks to its position, seeded arbitrary
    patterns (bits above M included) agree with the oracle's bisection, and
    the records per level are the distinct prefixes of the list."""
    st = OC.sector_enumerate(M, cons)
    s = mbr.sector_build(M, cons, width_bits=width)
    r = mbr.build_bitmap_trie(s, k)
    info = r.info()
    H = -(-M // k)
    assert info.kind == mbr.RANKER_BITMAP_TRIE and info.levels == H
    recs, rbytes, lds = mbr.bitmap_trie_levels(r)
    assert mbr.trie_bytes(r) == info.bytes >= sum(n * b for n, b in zip(recs, rbytes))
    widths = [M - (H - 1) * k] + [k] * (H - 1)
    above = M
    for l in range(H):
        above -= widths[l]                        # bits below and in chunk l
        pre = st >> np.uint64(above + widths[l]) if above + widths[l] < 64 else np.zeros_like(st)
        assert recs[l] == np.unique(pre).size, (l, recs[l])
        # one record size on every level, for the widest chunk: base, prefix
        # bytes of the map words (when there are several), the map; a power of two
        mw = -(-(1 << max(widths)) // 32)
        need = 4 * (1 + (-(-mw // 4) if mw > 1 else 0) + mw)
        assert rbytes[l] == max(8, 1 << int(np.ceil(np.log2(need))))
    dev = dev_u32 if width == 32 else dev_u64
    got = host_rank(mbr.rank_batch(r, dev(st)))
    assert np.array_equal(got, np.arange(st.size))
    lim = (1 << min(M + 1, 64)) - 1 if M < 64 else (1 << 64) - 1
    noise = synth.splitmix64(seed + M * 31 + k, n_noise) & np.uint64(lim)
    q = np.concatenate([noise, st[::max(1, st.size // 700)] ^ np.uint64(1)])
    if M < width:
        q = np.concatenate([q, st[: min(500, st.size)] | np.uint64(1 << M)])
    got = host_rank(mbr.rank_batch(r, dev(q)))
    assert np.array_equal(got, OC.bisect_rank(st, q))
    return r


@pytest.mark.parametrize("M,N,k", [(6, 2, 2), (12, 6, 1), (13, 5, 3), (16, 8, 4), (16, 8, 5), (17, 8, 6),
                                   (20, 10, 7), (24, 12, 8), (9, 0, 4), (9, 9, 4), (28, 1, 8)])
def test_bitmap_trie_particle_number_sectors(M, N, k):
    say("bitmap trie", M, N, k)
    _bt_check(M, OC.constraints(M, N), k)


@pytest.mark.parametrize("k", [3, 5, 8])
def test_bitmap_trie_irregular_and_wide(k):
    _bt_check(20, OC.constraints(20, 10, [(0xFF, 6, 8)]), k)
    _bt_check(18, [(0x3FFFF, 7, 9), (0x5555, 2, 5)], k)
    _bt_check(24, OC.spin_constraints(12, 6, 5), k)
    _bt_check(40, OC.constraints(40, 3, [(0xF, 1, 2)]), k, width=64)


@pytest.mark.parametrize("k", [4, 8])
def test_bitmap_trie_ras_m32_full_size(k):
    """The general-sector workload: M = 32, N = 16 with >= 6 of orbitals 0-7
    occupied (66,110,671 states), 2^24 queries, 90% members and 10% non-members
    (popcount 16, at most 5 of orbitals 0-7), as for the packed trie."""
    M = 32
    cons = OC.constraints(M, 16, [(0xFF, 6, 8)])
    st = OC.sector_enumerate(M, cons)
    s = mbr.sector_build(M, cons)
    r = mbr.build_bitmap_trie(s, k)
    say("ras bitmap trie k", k, "bytes", r.info().bytes, mbr.bitmap_trie_levels(r))
    nq = 1 << 24
    nm = nq // 10
    idx = synth.uniform_indices(3, nq - nm, st.size)
    pool = synth.random_subset_patterns(33, 3 * nm, 32, 16)
    low = np.array([bin(int(v) & 0xFF).count("1") for v in pool])
    non = pool[low <= 5][:nm]
    q = np.concatenate([st[idx], non])
    perm = synth.shuffle_positions(34, q.size)
    q = q[perm]
    want = np.concatenate([idx, np.full(nm, -1)])[perm]
    assert np.array_equal(host_rank(mbr.rank_batch(r, dev_u32(q))), want)


def test_bitmap_trie_rejects_bad_args():
    s = mbr.sector_build(10, OC.constraints(10, 5))
    for k in (0, 9):
        with pytest.raises(mbr.MbrError):
            mbr.build_bitmap_trie(s, k)
    e = mbr.sector_build(10, [((1 << 10) - 1, 4, 4), (0x3, 3, 3)])
    with pytest.raises(mbr.MbrError):
        mbr.build_bitmap_trie(e, 4)
