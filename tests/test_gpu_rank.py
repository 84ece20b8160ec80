"""GPU parity of sector enumeration, unrank, staggered and spin-resolved ranking
against the oracle (bit-exact)."""
import math

import numpy as np
import pytest

from oracle import combinatorics as OC
from oracle import staggered as OS
import synth
from tests._util import dev_u32, dev_u64, host_u32, host_u64, host_rank, say

pytestmark = pytest.mark.gpu

mbr = pytest.importorskip("paper_2203_04158_amd")


def _build(M, cons, width=32):
    return mbr.sector_build(M, cons, width_bits=width)


@pytest.mark.parametrize("M,cons", [
    (4, OC.constraints(4, 3)),
    (12, OC.constraints(12, 5)),
    (24, OC.constraints(24, 12)),
    (20, [(0xFF, 2, 5), (0xF0000, 1, 1)]),          # no fixed N: full scan
    (16, OC.constraints(16, 8, [(0xF, 3, 4)])),      # RAS-like
    (28, OC.spin_constraints(14, 7, 7)),             # spin product via disjoint windows
    (10, [((1 << 10) - 1, 4, 4), (0x3, 3, 3)]),      # empty sector
    (1, OC.constraints(1, 1)),
])
def test_sector_build(M, cons):
    say("sector", M, cons)
    want = OC.sector_enumerate(M, cons)
    s = _build(M, cons)
    assert s.size == want.size
    if want.size:
        assert np.array_equal(host_u32(s.states()), want)


def test_sector_build_u64():
    cons = OC.constraints(36, 3, [(0x7, 1, 2)])
    want = OC.sector_enumerate(36, cons)
    s = _build(36, cons, width=64)
    assert s.size == want.size
    assert np.array_equal(host_u64(s.states()), want)


def test_unrank_edges():
    s = _build(12, OC.constraints(12, 6))
    st = OC.sector_enumerate(12, OC.constraints(12, 6))
    idx = np.array([0, 1, st.size - 1, st.size, 2 ** 31, 0xFFFFFFFE], dtype=np.uint64)
    got = host_u32(mbr.unrank_batch(s, dev_u32(idx)))
    assert list(got[:3]) == [st[0], st[1], st[-1]]
    assert (got[3:] == 0xFFFFFFFF).all()
    import torch
    empty = torch.empty(0, dtype=torch.int32, device="cuda")
    assert mbr.unrank_batch(s, empty).numel() == 0


@pytest.mark.parametrize("M,N,k", [(24, 12, 8), (13, 6, 5), (32, 16, 8), (14, -1, 7), (9, 3, 16)])
def test_staggered_table_entries(M, N, k):
    r = mbr.build_staggered_tables(M, N, k)
    tab = mbr.staggered_table(r)
    nmax = M if N < 0 else N
    rows = OS.staggered_rows(M, k, nmax)
    assert tab.size == len(rows) << k
    for ri, (c, Mp, Np, w) in enumerate(rows):
        for v in range(1 << w):
            assert tab[(ri << k) + v] == OS.partrank(v, Mp, Np)


def test_staggered_cfg1_all_members_and_queries():
    M, N, k = 24, 12, 8
    st = OC.sector_enumerate(M, OC.constraints(M, N))
    r = mbr.build_staggered_tables(M, N, k)
    got = host_rank(mbr.rank_batch(r, dev_u32(st)))
    assert np.array_equal(got, np.arange(st.size))
    # 2^22 seeded uniform queries, as in the ranking microbenchmark
    idx = synth.uniform_indices(1, 1 << 22, st.size)
    q = st[idx]
    got = host_rank(mbr.rank_batch(r, dev_u32(q)))
    assert np.array_equal(got, OC.bisect_rank(st, q))
    # non-members: wrong popcount, bits at or above M
    bad = np.concatenate([synth.splitmix64(5, 100000) & np.uint64(0xFFFFFFFF),
                          st[:1000] | np.uint64(1 << 24)])
    got = host_rank(mbr.rank_batch(r, dev_u32(bad)))
    assert np.array_equal(got, OC.bisect_rank(st, bad))


@pytest.mark.parametrize("M,N,k", [(13, 6, 1), (13, 6, 3), (17, 9, 5), (20, 3, 11), (32, 16, 16),
                                   (32, 1, 8), (32, 31, 4), (16, 0, 8), (16, 16, 8)])
def test_staggered_against_cns(M, N, k):
    q = synth.random_subset_patterns(M * 100 + N, 50000, M, N)
    noise = synth.splitmix64(M + 7 * N, 20000) & np.uint64((1 << M) - 1)
    q = np.concatenate([q, noise])
    r = mbr.build_staggered_tables(M, N, k)
    got = host_rank(mbr.rank_batch(r, dev_u32(q)))
    pc = np.array([bin(int(a)).count("1") for a in q])
    want = np.where(pc == N, OC.cns_rank_batch(q).astype(np.int64), -1)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("M,N,k", [(40, 20, 8), (64, 32, 8), (64, 5, 13), (48, 24, 16), (64, 32, 16),
                                   (64, 63, 4), (50, 25, 7)])
def test_staggered_u64(M, N, k):
    """64-bit patterns; sectors of 2^32 states or more rank through the 64-bit
    entry point (the 32-bit one refuses them), against Eq. cns on the host."""
    import torch
    q = synth.random_subset_patterns(M + N + k, 40000, M, N)
    noise = synth.splitmix64(M * 3 + k, 20000)
    if M < 64:
        noise &= np.uint64((1 << M) - 1)
    q = np.concatenate([q, noise])
    pc = np.array([bin(int(a)).count("1") for a in q])
    inw = (q >> np.uint64(M)) == 0 if M < 64 else np.ones(q.size, bool)
    member = (pc == N) & inw
    r = mbr.build_staggered_tables(M, N, k, width_bits=64)
    want64 = np.where(member, OC.cns_rank_batch(q), np.uint64(0xFFFFFFFFFFFFFFFF))
    got64 = mbr.rank_batch64(r, dev_u64(q)).cpu().numpy().view(np.uint64)
    assert np.array_equal(got64, want64)
    if math.comb(M, N) >= 2 ** 32 - 1:
        with pytest.raises(mbr.MbrError):
            mbr.rank_batch(r, dev_u64(q))
    else:
        got = host_rank(mbr.rank_batch(r, dev_u64(q)))
        assert np.array_equal(got, np.where(member, OC.cns_rank_batch(q).astype(np.int64), -1))
    # unaligned 64-bit rank output, ragged length
    out = torch.zeros(q.size + 1, dtype=torch.int64, device="cuda")[1:]
    mbr.rank_batch64(r, dev_u64(q), out=out)
    assert np.array_equal(out.cpu().numpy().view(np.uint64), want64)


@pytest.mark.parametrize("L,nu,nd,k", [(14, 7, 7, 7), (14, 7, 7, 14), (12, 3, 8, 5), (4, 1, 2, 2),
                                       (12, 0, 12, 6), (16, 4, 5, 8)])
def test_spin_ranker(L, nu, nd, k):
    st = OC.sector_enumerate(2 * L, OC.spin_constraints(L, nu, nd))
    r = mbr.build_spin_ranker(L, nu, nd, k)
    got = host_rank(mbr.rank_batch(r, dev_u32(st)))
    assert np.array_equal(got, np.arange(st.size))
    bad = synth.splitmix64(L * 31 + nu, 50000) & np.uint64((1 << min(32, 2 * L + 1)) - 1)
    got = host_rank(mbr.rank_batch(r, dev_u32(bad)))
    assert np.array_equal(got, OC.bisect_rank(st, bad))


@pytest.mark.parametrize("kind", ["stag32", "stag64", "spin"])
@pytest.mark.parametrize("qoff,ooff,n", [(0, 0, 1), (0, 0, 4097), (1, 0, 4099), (0, 3, 10001),
                                         (2, 1, 70001), (0, 0, 0), (0, 0, 1 << 20)])
def test_rank_ragged_and_unaligned(kind, qoff, ooff, n):
    """Vector (16-byte) and scalar access paths: sizes with a ragged tail, and
    query / output views that start off the vector alignment."""
    import torch
    if kind == "spin":
        L, nu, nd = 12, 5, 6
        st = OC.sector_enumerate(2 * L, OC.spin_constraints(L, nu, nd))
        r = mbr.build_spin_ranker(L, nu, nd, 6)
        lim, dev = (1 << (2 * L)) - 1, dev_u32
    else:
        M, N = (22, 9) if kind == "stag32" else (40, 4)
        st = OC.sector_enumerate(M, OC.constraints(M, N)) if M <= 32 else None
        r = mbr.build_staggered_tables(M, N, 7, width_bits=32 if M <= 32 else 64)
        lim, dev = (1 << M) - 1, (dev_u32 if M <= 32 else dev_u64)
    if st is not None:
        idx = synth.uniform_indices(n + 5, n + qoff, st.size) if n + qoff else np.zeros(0, np.int64)
        q = st[idx]
        q[::7] = synth.splitmix64(n + 9, q[::7].size) & np.uint64(lim)  # non-members mixed in
        want = OC.bisect_rank(st, q)
    else:
        q = synth.random_subset_patterns(n + 11, n + qoff, 40, 4) if n + qoff else np.zeros(0, np.uint64)
        q[::5] = synth.splitmix64(n + 3, q[::5].size) & np.uint64(lim)
        pc = np.array([bin(int(a)).count("1") for a in q], dtype=np.int64)
        want = np.where(pc == 4, OC.cns_rank_batch(q).astype(np.int64), -1)
    qd = dev(q)[qoff:]
    out = torch.full((n + ooff,), 7, dtype=torch.int32, device="cuda")[ooff:]
    mbr.rank_batch(r, qd, out=out)
    assert np.array_equal(host_rank(out), want[qoff:])


@pytest.mark.parametrize("L,nu,nd", [(6, 3, 2), (6, 0, 6), (6, 6, 0), (1, 1, 0), (12, 5, 6),
                                     (14, 7, 7), (17, 3, 4), (19, 1, 9), (20, 2, 3)])
def test_unrank_spin_matches_sector_list(L, nu, nd):
    """Every index of the spin sector (L <= 16: half lists in LDS; L > 16:
    greedy combinadics) against the oracle's ascending sector list, plus
    indices past the end."""
    st = OC.sector_enumerate(2 * L, OC.spin_constraints(L, nu, nd))
    r = mbr.build_spin_ranker(L, nu, nd, min(L, 8))
    wide = 2 * L > 32
    idx = np.concatenate([np.arange(st.size, dtype=np.uint64),
                          np.array([st.size, st.size + 1, 0xFFFFFFFE], dtype=np.uint64)])
    out = mbr.unrank_spin_batch(r, dev_u32(idx))
    got = host_u64(out) if wide else host_u32(out)
    ones = np.uint64(0xFFFFFFFFFFFFFFFF if wide else 0xFFFFFFFF)
    assert np.array_equal(got[:st.size], st)
    assert (got[st.size:] == ones).all()


def test_unrank_spin_l16_full_size_round_trip():
    """(8,8) on 16 sites (165,636,900 states, no list stored): 2^22 uniform
    indices; each pattern has the sector's popcounts, ranks back to its index
    on the GPU, and sampled ones match the oracle's combinadics of each half
    composed by Eq. rankupdown."""
    L, nu, nd = 16, 8, 8
    n_dn = OC.binom(L, nd)
    total = OC.binom(L, nu) * n_dn
    r = mbr.build_spin_ranker(L, nu, nd, 8)
    idx = synth.uniform_indices(7, 1 << 22, total).astype(np.uint64)
    idx[:3] = [0, total - 1, total // 2]
    pat = mbr.unrank_spin_batch(r, dev_u32(idx))
    back = host_rank(mbr.rank_batch(r, pat))
    assert np.array_equal(back, idx.astype(np.int64))
    p = host_u32(pat)
    lo, hi = p & np.uint64(0xFFFF), p >> np.uint64(16)
    pc = lambda v: np.array([bin(int(t)).count("1") for t in v[:4096]])
    assert (pc(lo) == nd).all() and (pc(hi) == nu).all()
    for t in range(0, 4096, 37):
        i = int(idx[t])
        assert OC.cns_rank(int(hi[t])) * n_dn + OC.cns_rank(int(lo[t])) == i


def test_unrank_spin_l32_sampled():
    """64-bit patterns on 32 sites, (3,2): sampled indices against the oracle's
    Eq. unrank of each half composed by Eq. rankupdown."""
    L, nu, nd = 32, 3, 2
    n_dn = OC.binom(L, nd)
    total = OC.binom(L, nu) * n_dn
    r = mbr.build_spin_ranker(L, nu, nd, 8)
    idx = synth.uniform_indices(11, 3000, total).astype(np.uint64)
    idx[:2] = [0, total - 1]
    got = host_u64(mbr.unrank_spin_batch(r, dev_u32(idx)))
    for t, i in enumerate(idx):
        i = int(i)
        want = (OC.cns_unrank(i // n_dn, nu, L) << L) | OC.cns_unrank(i % n_dn, nd, L)
        assert int(got[t]) == want, (i, hex(int(got[t])), hex(want))


def test_unrank_spin_rejects_other_rankers():
    r = mbr.build_staggered_tables(12, 6, 6)
    with pytest.raises(mbr.MbrError):
        mbr.unrank_spin_batch(r, dev_u32(np.arange(4, dtype=np.uint64)))


@pytest.mark.parametrize("L,nu,nd", [(12, 5, 6), (18, 2, 3)])
@pytest.mark.parametrize("qoff,ooff,n", [(0, 0, 1), (0, 0, 4099), (1, 0, 4097), (0, 3, 10001),
                                         (2, 1, 70001), (0, 0, 1 << 20)])
def test_unrank_spin_ragged_and_unaligned(L, nu, nd, qoff, ooff, n):
    """Vector (16-byte) and scalar access paths: sizes with a ragged tail, and
    index / output views that start off the vector alignment."""
    import torch
    st = OC.sector_enumerate(2 * L, OC.spin_constraints(L, nu, nd))
    r = mbr.build_spin_ranker(L, nu, nd, 6)
    idx = synth.uniform_indices(n + qoff, n, st.size + 5).astype(np.uint64)  # a few past the end
    qbuf = dev_u32(np.concatenate([np.zeros(qoff, np.uint64), idx]))
    wide = 2 * L > 32
    obuf = torch.empty(n + ooff, dtype=torch.int64 if wide else torch.int32, device="cuda")
    mbr.unrank_spin_batch(r, qbuf[qoff:], out=obuf[ooff:])
    got = host_u64(obuf[ooff:]) if wide else host_u32(obuf[ooff:])
    ones = np.uint64(0xFFFFFFFFFFFFFFFF if wide else 0xFFFFFFFF)
    inside = idx < st.size
    assert np.array_equal(got[inside], st[idx[inside]])
    assert (got[~inside] == ones).all()


def test_binding_rejects_wrong_buffers():
    """The C ABI takes raw pointers; the binding checks element size, device
    and length before any launch."""
    import torch
    r = mbr.build_staggered_tables(12, 6, 6)
    q = dev_u32(np.arange(100, dtype=np.uint64))
    with pytest.raises(ValueError):
        mbr.rank_batch(r, q.long())                                   # 8-byte queries for a 32-bit ranker
    with pytest.raises(ValueError):
        mbr.rank_batch(r, q, out=torch.empty(99, dtype=torch.int32, device="cuda"))   # short output
    with pytest.raises(ValueError):
        mbr.rank_batch(r, q.cpu())                                    # host tensor
    s = mbr.sector_build(12, OC.constraints(12, 6))
    with pytest.raises(ValueError):
        mbr.unrank_batch(s, q, out=torch.empty(100, dtype=torch.int64, device="cuda"))
    h = mbr.hubbard_create(4, [(0, 1, 1.0), (1, 2, 1.0)], [(2, 2)], U=[1.0] * 4)
    x = torch.zeros(h.dim, dtype=torch.float32, device="cuda")      # fp64 Hamiltonian
    with pytest.raises(ValueError):
        mbr.hubbard_apply(h, x, torch.empty_like(x))
    x = torch.zeros(h.dim - 1, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        mbr.hubbard_apply(h, x, torch.zeros(h.dim, dtype=torch.float64, device="cuda"))
