"""Rank-side autotuning: the chunk width k picked per ranker kind and sector,
the learned ranker's window-or-fallback choice, and the trie width of the
trie-ranked H·x.  Whatever is picked, the ranks must stay exact (against the
oracle's bisection on its own enumeration) and the product bitwise equal to
the staggered-halves product."""
import numpy as np
import pytest

from oracle import combinatorics as OC
from oracle import hamiltonian as OH
import synth
from tests._util import dev_u32, dev_u64, host_rank, say

pytestmark = pytest.mark.gpu
mbr = pytest.importorskip("paper_2203_04158_amd")
torch = pytest.importorskip("torch")


def _queries(st, M, seed, n_noise=30000):
    noise = synth.splitmix64(seed, n_noise) & np.uint64((1 << M) - 1)
    members = st[synth.uniform_indices(seed + 1, 60000, st.size)]
    return np.concatenate([members, noise])


@pytest.mark.parametrize("kind,ks", [(1, None), (3, [4, 8, 10]), (8, None)])
def test_rank_autotune_picks_a_candidate_and_ranks_exactly(kind, ks, tmp_path, monkeypatch):
    M = 20
    cons = OC.constraints(M, 10) if kind == 1 else OC.constraints(M, 10, [(0xFF, 4, 6)])
    st = OC.sector_enumerate(M, cons)
    s = mbr.sector_build(M, cons)
    q = _queries(st, M, seed=kind * 11)
    qd = dev_u32(q)
    cache = tmp_path / "tune.txt"
    cache.write_text("rank;garbage\nnot a line at all\n")
    monkeypatch.setenv("MBR_AUTOTUNE_CACHE", str(cache))
    r, t = mbr.rank_autotune(s, kind, qd, ks=ks, reps=2)
    say("rank autotune kind", kind, t)
    default = {1: [3, 4, 5, 6, 7, 8, 10, 12, 14, 16], 3: [4, 6, 8, 10, 12], 8: [4, 5, 6, 7, 8]}[kind]
    cand = sorted(set(min(k, M) for k in (ks or default)))
    assert t["kind"] == kind and t["k"] in cand and not t["from_cache"]
    assert t["tried"] == len(cand) and t["ms"] > 0
    assert r.info().kind == kind and r.info().k == t["k"]
    want = OC.bisect_rank(st, q)
    assert np.array_equal(host_rank(mbr.rank_batch(r, qd)), want)
    # the second call is served from the cache with the same width
    assert len(cache.read_text().splitlines()) == 3
    r2, t2 = mbr.rank_autotune(s, kind, qd, ks=ks, reps=2)
    assert t2["from_cache"] and t2["k"] == t["k"] and t2["tried"] == 0
    assert np.array_equal(host_rank(mbr.rank_batch(r2, qd)), want)
    assert len(cache.read_text().splitlines()) == 3


@pytest.mark.parametrize("kind", [1, 3, 8])
def test_rank_autotune_64_bit_patterns(kind):
    """M = 40 with 64-bit patterns (three particles, one or two of them in
    orbitals 0-3 for the tries, three anywhere for the staggered tables):
    whatever width is picked, the ranks equal the oracle's bisection."""
    M = 40
    cons = OC.constraints(M, 3) if kind == 1 else OC.constraints(M, 3, [(0xF, 1, 2)])
    st = OC.sector_enumerate(M, cons)
    s = mbr.sector_build(M, cons, width_bits=64)
    noise = synth.splitmix64(91, 20000) & np.uint64((1 << M) - 1)
    q = np.concatenate([st[synth.uniform_indices(92, 30000, st.size)], noise])
    qd = dev_u64(q)
    r, t = mbr.rank_autotune(s, kind, qd, ks=[4, 6, 8], reps=2)
    say("rank autotune, 64-bit patterns, kind", kind, t)
    assert t["k"] in (4, 6, 8) and t["tried"] == 3
    assert np.array_equal(host_rank(mbr.rank_batch(r, qd)), OC.bisect_rank(st, q))


def test_rank_autotune_rejects():
    M = 16
    ras = mbr.sector_build(M, OC.constraints(M, 8, [(0xF, 1, 2)]))
    q = dev_u32(np.arange(64, dtype=np.uint64))
    with pytest.raises(mbr.MbrError):   # staggered tables need a plain C(M, N) sector
        mbr.rank_autotune(ras, mbr.RANKER_STAGGERED, q)
    with pytest.raises(mbr.MbrError):   # not a tunable kind
        mbr.rank_autotune(ras, mbr.RANKER_LEARNED, q)
    with pytest.raises(mbr.MbrError):   # bitmap tries take k <= 8
        mbr.rank_autotune(ras, mbr.RANKER_BITMAP_TRIE, q, ks=[4, 9])
    with pytest.raises(mbr.MbrError):
        mbr.rank_autotune(ras, mbr.RANKER_TRIE, q, reps=0)


def test_learned_autotune_keeps_the_faster_path_and_exact_ranks():
    M, cons = 20, OC.constraints(20, 10)
    st = OC.sector_enumerate(M, cons)
    s = mbr.sector_build(M, cons)
    trie = mbr.build_trie(s, 8)
    lr_ = mbr.learned_train(s, trie, epochs=10, batch=4096, lr=3e-3, seed=1, max_window=1 << 20)
    q = _queries(st, M, seed=5)
    qd = dev_u32(q)
    tw, tf = mbr.learned_autotune(lr_, qd, reps=3)
    _, win = mbr.learned_max_error(lr_)
    say("learned window", tw, "ms, fallback", tf, "ms, window serves:", win)
    assert tw > 0 and tf > 0 and win == (tw <= tf)
    assert np.array_equal(host_rank(mbr.rank_batch(lr_, qd)), OC.bisect_rank(st, q))
    with pytest.raises(mbr.MbrError):
        mbr.learned_autotune(trie, qd)


def test_trie_ranked_hubbard_autotune_width():
    L = 8
    bonds = OH.chain_bonds(L) + [(0, 3, 0.4)]
    sectors = [(4, 4), (3, 5), (2, 1)]
    U = [2.5] * L
    hs = mbr.hubbard_create(L, bonds, sectors, U=U)
    ht = mbr.hubbard_create(L, bonds, sectors, U=U, rank_kind=mbr.RANK_TRIE)
    assert mbr.hubbard_get_config(ht)["k"] == 4           # default: four levels over 16-bit patterns
    cfg = mbr.hubbard_autotune(ht, reps=2)
    say("trie-ranked H·x autotune", cfg)
    assert cfg["k"] in (4, 6, 8) and cfg["tuned_ms"] > 0
    x = torch.from_numpy(2 * synth.uniform01(17, hs.dim) - 1).cuda()
    y1, y2 = torch.empty_like(x), torch.empty_like(x)
    mbr.hubbard_apply(hs, x, y1)
    mbr.hubbard_apply(ht, x, y2)
    assert torch.equal(y1, y2)
    # every width gives the same product
    for k in (4, 6, 8):
        hk = mbr.hubbard_create(L, bonds, sectors, U=U, rank_kind=mbr.RANK_TRIE, k=k)
        assert mbr.hubbard_get_config(hk)["k"] == k
        yk = torch.empty_like(x)
        mbr.hubbard_apply(hk, x, yk)
        assert torch.equal(y1, yk)
