"""GPU parity of the learned index: network forward and gradients against the
fp64 oracle, and exactness of learned ranking.

Forward bound: the matrix-core path rounds each hidden activation to bf16
(relative error <= 2^-9) and accumulates in fp32, so with the oracle's fp64
intermediates h1, h2 (same bf16-rounded weights)
  |y_gpu - y| <= 2^-8 * sum_j |w3_j| (sum_k |W2_jk| h1_k + h2_j) + 2^-16 * scale.
Gradient bound: training keeps activations in fp32 (bf16 weights only), so the
gradients agree with the fp64 oracle to fp32 accumulation error over the
batch; the test uses 1e-4 of each tensor's largest entry.
"""
import numpy as np
import pytest

from oracle import combinatorics as OC
from oracle import mlp as OM
import synth
from tests._util import dev_u32, host_rank, say

pytestmark = pytest.mark.gpu
mbr = pytest.importorskip("paper_2203_04158_amd")
torch = pytest.importorskip("torch")


def _bf16(a):
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _split(flat):
    f = np.asarray(flat, dtype=np.float64)
    return [f[0:2048].reshape(64, 32), f[2048:2112], f[2112:6208].reshape(64, 64),
            f[6208:6272], f[6272:6336], float(f[6336])]


def _random_params(seed, scale=1.0):
    u = 2 * synth.uniform01(seed, 6337) - 1
    u[:2048] *= 0.4 * scale
    u[2048:2112] *= 0.1
    u[2112:6208] *= 0.25 * scale
    u[6208:6272] *= 0.1
    u[6272:6336] *= 0.3
    return u.astype(np.float32)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_forward_matches_oracle(seed):
    B = 2048
    p32 = _random_params(seed)
    q = (synth.splitmix64(seed + 100, B) & np.uint64(0xFFFFFFFF))
    q[:4] = [0, 0xFFFFFFFF, 1, 1 << 31]
    y = mbr.mlp_forward(torch.from_numpy(p32).cuda(), dev_u32(q)).cpu().numpy().astype(np.float64)
    P = _split(_bf16(p32))
    X = OM.features(q)
    want, (X_, z1, h1, z2, h2) = OM.forward(P, X)
    W1, b1, W2, b2, w3, b3 = P
    bound = 2.0 ** -8 * (np.abs(w3) * (h1 @ np.abs(W2).T + h2)).sum(axis=1)
    bound += 2.0 ** -16 * (1 + np.abs(want))
    err = np.abs(y - want)
    assert (err <= bound).all(), (err.max(), bound[err.argmax()])


@pytest.mark.parametrize("seed", [4, 5])
def test_gradients_match_oracle(seed):
    B = 512
    p32 = _random_params(seed)
    q = synth.splitmix64(seed + 7, B) & np.uint64(0xFFFFFF)
    tgt = synth.uniform01(seed + 9, B).astype(np.float32)
    g, loss = mbr.mlp_gradients(torch.from_numpy(p32).cuda(), dev_u32(q), torch.from_numpy(tgt).cuda())
    g = g.cpu().numpy().astype(np.float64)
    P = _split(_bf16(p32))
    X = OM.features(q)
    G = OM.gradients(P, X, tgt.astype(np.float64))
    want_loss = OM.loss(P, X, tgt.astype(np.float64))
    assert abs(float(loss.cpu()[0]) - want_loss) <= 1e-5 * max(1.0, want_loss)
    got = _split(g)
    for name, a, b in zip(["W1", "b1", "W2", "b2", "w3", "b3"], got, G):
        a = np.atleast_1d(a)
        b = np.atleast_1d(b)
        tol = 1e-4 * max(1e-12, np.abs(b).max())
        assert np.abs(a - b).max() <= tol, (name, np.abs(a - b).max(), tol)


def _learned(M, cons, epochs, batch=4096, lr=3e-3, max_window=1 << 20, k=8, seed=1):
    s = mbr.sector_build(M, cons)
    trie = mbr.build_trie(s, k)
    lr_ = mbr.learned_train(s, trie, epochs=epochs, batch=batch, lr=lr, seed=seed,
                            max_window=max_window)
    return s, trie, lr_


def _leaf_windows(y, nleaf, n):
    """Stage-2 windows recomputed on the host from the network outputs y of the
    members 0..n-1 (same leaf rule as the library: floor(y nleaf) in fp32,
    clamped, NaN and y <= 0 to leaf 0)."""
    yf = np.asarray(y, dtype=np.float32)
    with np.errstate(invalid="ignore"):
        b = np.where(~(yf > 0), 0, np.where(yf >= 1, nleaf - 1,
                     np.floor(yf * np.float32(nleaf)))).astype(np.int64)
    lo = np.full(nleaf, np.iinfo(np.int64).max)
    hi = np.full(nleaf, -1)
    np.minimum.at(lo, b, np.arange(n))
    np.maximum.at(hi, b, np.arange(n))
    return b, lo, hi


def test_learned_ranks_exact_and_error_recorded():
    M, cons = 20, OC.constraints(20, 10)
    st = OC.sector_enumerate(M, cons)
    s, trie, lr_ = _learned(M, cons, epochs=30)
    e, win = mbr.learned_max_error(lr_)
    info = mbr.learned_stats(lr_)
    assert win and info["uses_window"] and info["max_window"] == e
    got = host_rank(mbr.rank_batch(lr_, dev_u32(st)))
    assert np.array_equal(got, np.arange(st.size))
    noise = synth.splitmix64(77, 50000) & np.uint64((1 << 21) - 1)
    got = host_rank(mbr.rank_batch(lr_, dev_u32(noise)))
    assert np.array_equal(got, OC.bisect_rank(st, noise))
    # the recorded windows are those of the query-time network
    params = torch.from_numpy(mbr.learned_params(lr_)).cuda()
    y = mbr.mlp_forward(params, dev_u32(np.concatenate([st, np.zeros((-st.size) % 64, np.uint64)])))
    y = y.cpu().numpy()[: st.size]
    nl = info["n_leaves"]
    # automatic: about four members per leaf, between 2^8 and 2^12 leaves
    assert nl == min(1 << 12, max(256, 1 << (st.size // 4 - 1).bit_length()))
    b, lo, hi = _leaf_windows(y, nl, st.size)
    assert int((hi - lo)[hi >= 0].max()) == e
    assert abs(info["mean_window"] - float((hi[b] - lo[b] + 1).mean())) <= 1e-9 * info["mean_window"]
    p = np.clip(np.rint(st.size * y.astype(np.float64)), 0, st.size - 1)
    assert int(np.abs(p - np.arange(st.size)).max()) == info["single_window_error"]
    say("learned M=20 N=10: leaf windows max", e, "mean", info["mean_window"],
        "single-window error", info["single_window_error"], "of", st.size)


def test_training_gain_over_untrained_network():
    """What training buys: the stage-2 windows of the untrained network are
    far wider than those of the trained one, and so is stage 1's own error."""
    M, cons = 20, OC.constraints(20, 10)
    _, _, untrained = _learned(M, cons, epochs=0)
    _, _, trained = _learned(M, cons, epochs=30)
    u, t = mbr.learned_stats(untrained), mbr.learned_stats(trained)
    say("untrained", u, "trained", t)
    assert t["mean_window"] * 10 < u["mean_window"]
    assert t["max_window"] * 10 < u["max_window"]
    assert t["single_window_error"] * 10 < u["single_window_error"]


def test_single_particle_sector_learns_exactly():
    # N = 1: rank(2^c) = c is linear in the features; training reaches e = 0
    M = 32
    cons = OC.constraints(M, 1)
    st = OC.sector_enumerate(M, cons)
    s, trie, lr_ = _learned(M, cons, epochs=3000, batch=256, lr=1e-2)
    e, win = mbr.learned_max_error(lr_)
    say("N=1 e", e)
    assert e == 0
    assert np.array_equal(host_rank(mbr.rank_batch(lr_, dev_u32(st))), np.arange(M))


def test_fallback_when_window_too_wide():
    M, cons = 16, OC.constraints(16, 8, [(0xF, 3, 4)])
    st = OC.sector_enumerate(M, cons)
    s, trie, lr_ = _learned(M, cons, epochs=0, max_window=0)
    e, win = mbr.learned_max_error(lr_)
    assert not win and e > 0
    q = np.concatenate([st, synth.splitmix64(3, 5000) & np.uint64(0xFFFF)])
    assert np.array_equal(host_rank(mbr.rank_batch(lr_, dev_u32(q))), OC.bisect_rank(st, q))


def test_training_is_repeatable():
    M, cons = 14, OC.constraints(14, 7)
    _, _, a = _learned(M, cons, epochs=5, seed=9)
    _, _, b = _learned(M, cons, epochs=5, seed=9)
    assert np.array_equal(mbr.learned_params(a), mbr.learned_params(b))
    assert mbr.learned_max_error(a) == mbr.learned_max_error(b)


def test_learned_chain_sector_full_size():
    """The (7,7) chain sector as 28-bit patterns (11,778,624 states), trained
    as in the ranking benchmark, with the window search forced (max_window
    above any leaf window): every member ranks to its index and seeded
    arbitrary 28-bit patterns agree with bisection on the oracle's list."""
    M, cons = 28, OC.spin_constraints(14, 7, 7)
    s = mbr.sector_build(M, cons)
    trie = mbr.build_trie(s, 8)
    lr_ = mbr.learned_train(s, trie, epochs=8, batch=4096, lr=2e-3, seed=4,
                            samples_per_epoch=1 << 22, max_window=1 << 30)
    info = mbr.learned_stats(lr_)
    say("chain sector learned", info)
    assert info["uses_window"] and info["max_window"] < s.size
    idx = torch.arange(s.size, dtype=torch.int32, device="cuda")
    got = mbr.rank_batch(lr_, s.states())
    assert torch.equal(got, idx)
    st = OC.sector_enumerate(M, cons)
    noise = synth.splitmix64(78, 1 << 20) & np.uint64((1 << 28) - 1)
    q = np.concatenate([noise, st[synth.uniform_indices(79, 1 << 20, st.size)]])
    assert np.array_equal(host_rank(mbr.rank_batch(lr_, dev_u32(q))), OC.bisect_rank(st, q))


@pytest.mark.parametrize("M,N", [(17, 1), (10, 4), (11, 4), (12, 5), (16, 3)])
def test_learned_ranks_exact_on_small_and_ragged_sectors(M, N):
    """Sector sizes 17, 210, 330, 792 and 560: not multiples of the 16- and
    256-state sampling strides, windows that start and end anywhere; every
    member and random non-members against the oracle."""
    cons = OC.constraints(M, N)
    st = OC.sector_enumerate(M, cons)
    s, trie, lr_ = _learned(M, cons, epochs=4, batch=256)
    got = host_rank(mbr.rank_batch(lr_, dev_u32(st)))
    assert np.array_equal(got, np.arange(st.size))
    noise = synth.splitmix64(M * 7 + N, 20000) & np.uint64((1 << (M + 1)) - 1)
    got = host_rank(mbr.rank_batch(lr_, dev_u32(noise)))
    assert np.array_equal(got, OC.bisect_rank(st, noise))


@pytest.mark.parametrize("M,N", [(1, 1), (17, 1), (10, 4), (11, 4), (12, 5), (16, 3), (20, 10)])
def test_sampled_search_ranks_exact(M, N):
    """The search without the network (whole list as the window): sector sizes
    1, 17, 210, 330, 792, 560 and 184,756 cover one to four sampled copies,
    ragged last lines and the bisection tail; every member and seeded
    non-members (bits above M included) against the oracle's bisection."""
    cons = OC.constraints(M, N)
    st = OC.sector_enumerate(M, cons)
    s = mbr.sector_build(M, cons)
    r = mbr.build_sampled_ranker(s)
    info = r.info()
    assert info.kind == mbr.RANKER_SAMPLED and info.n_states == st.size
    got = host_rank(mbr.rank_batch(r, dev_u32(st)))
    assert np.array_equal(got, np.arange(st.size))
    noise = synth.splitmix64(M * 11 + N, 30001) & np.uint64((1 << min(M + 1, 32)) - 1)
    got = host_rank(mbr.rank_batch(r, dev_u32(noise)))
    assert np.array_equal(got, OC.bisect_rank(st, noise))


def test_sampled_search_chain_sector_and_rejects():
    """Full-size (7,7) chain sector (11,778,624 states, three sampled copies):
    every member, and 2^20 seeded 28-bit patterns against the oracle; 64-bit
    sectors are refused."""
    M, cons = 28, OC.spin_constraints(14, 7, 7)
    s = mbr.sector_build(M, cons)
    r = mbr.build_sampled_ranker(s)
    idx = torch.arange(s.size, dtype=torch.int32, device="cuda")
    assert torch.equal(mbr.rank_batch(r, s.states()), idx)
    st = OC.sector_enumerate(M, cons)
    noise = synth.splitmix64(91, 1 << 20) & np.uint64((1 << 28) - 1)
    assert np.array_equal(host_rank(mbr.rank_batch(r, dev_u32(noise))), OC.bisect_rank(st, noise))
    s64 = mbr.sector_build(40, OC.constraints(40, 1), width_bits=64)
    with pytest.raises(mbr.MbrError):
        mbr.build_sampled_ranker(s64)


def test_leaf_count_option():
    """An explicit 2^b leaves is honoured (ranks stay exact); b outside 8..28
    is refused."""
    M, cons = 12, OC.constraints(12, 5)
    st = OC.sector_enumerate(M, cons)
    s = mbr.sector_build(M, cons)
    trie = mbr.build_trie(s, 4)
    for b in (8, 11):
        r = mbr.learned_train(s, trie, epochs=2, batch=256, lr=3e-3, seed=2, max_window=1 << 20,
                              log2_leaves=b)
        assert mbr.learned_stats(r)["n_leaves"] == 1 << b
        assert np.array_equal(host_rank(mbr.rank_batch(r, dev_u32(st))), np.arange(st.size))
    for b in (7, 29, -1):
        with pytest.raises(mbr.MbrError):
            mbr.learned_train(s, trie, epochs=1, batch=256, log2_leaves=b)


def _m32_8x8_list():
    """The sector M = 32 with 8 particles in each 16-bit half (165,636,900
    states), ascending.  Its members are the pairs (upper half, lower half) of
    two 8-of-16 patterns, and ascending order is the order of the upper half,
    then of the lower; the list is built that way from the oracle's 16-bit
    sector and checked against the oracle's enumeration at M = 20."""
    def pairs(h):
        half = OC.sector_enumerate(h, OC.constraints(h, h // 2))
        return ((half[:, None] << np.uint64(h)) | half[None, :]).ravel()
    small = pairs(10)
    assert np.array_equal(small, OC.sector_enumerate(20, OC.spin_constraints(10, 5, 5)))
    st = pairs(16)
    assert st.size == 12870 ** 2
    return st


@pytest.mark.timeout(900)
def test_learned_and_sampled_m32_8x8_full_size():
    """Ranking config 4(b): M = 32, N_up = N_dn = 8 (165,636,900 states; four
    sampled copies and bit 31 in use), trained as in the benchmark with the
    window search forced.  Every member ranks to its index, and 2^20 uniform
    members plus 2^20 arbitrary 32-bit patterns agree with bisection on the
    oracle's list, for the learned ranker and for the same search without the
    network."""
    M, cons = 32, OC.spin_constraints(16, 8, 8)
    st = _m32_8x8_list()
    s = mbr.sector_build(M, cons)
    assert s.size == st.size
    states = s.states()
    assert np.array_equal(states.cpu().numpy().view(np.uint32), st.astype(np.uint32))
    sampled = mbr.build_sampled_ranker(s)
    lr_ = mbr.learned_train(s, sampled, epochs=8, batch=4096, lr=2e-3, seed=4,
                            samples_per_epoch=1 << 22, max_window=1 << 31)
    info = mbr.learned_stats(lr_)
    say("m32 8+8 learned", info, "sampled levels", sampled.info().levels)
    assert info["uses_window"]
    idx = torch.arange(s.size, dtype=torch.int32, device="cuda")
    noise = synth.splitmix64(80, 1 << 20) & np.uint64(0xFFFFFFFF)
    noise[:4] = [0, 0xFFFFFFFF, 1 << 31, 0xFF00FF00]
    q = np.concatenate([st[synth.uniform_indices(81, 1 << 20, st.size)], noise])
    want = OC.bisect_rank(st, q)
    for name, r in (("learned", lr_), ("sampled", sampled)):
        say("m32 8+8 all members:", name)
        assert torch.equal(mbr.rank_batch(r, states), idx), name
        assert np.array_equal(host_rank(mbr.rank_batch(r, dev_u32(q))), want), name


def test_learned_windows_narrow_the_search():
    """What the trained network gains over the same search without it, in
    probes: the search narrows a window by 16x per sampled level, so a window
    of w states needs ceil(log16 w) levels and the whole list
    ceil(log16 N_s).  On the (7,7) chain sector, trained as in the benchmark,
    the members' own leaf windows (recomputed on the host from the query-time
    network outputs) save at least half a level on average and are at least
    ten times narrower than the list.  Throughput is the bench's business:
    there the network's forward pass costs more than the saved levels."""
    M, cons = 28, OC.spin_constraints(14, 7, 7)
    s = mbr.sector_build(M, cons)
    sampled = mbr.build_sampled_ranker(s)
    lr_ = mbr.learned_train(s, sampled, epochs=8, batch=4096, lr=2e-3, seed=4,
                            samples_per_epoch=1 << 22, max_window=1 << 31)
    info = mbr.learned_stats(lr_)
    st = s.states()
    n = s.size
    pad = (-n) % 64
    q = torch.cat([st, torch.zeros(pad, dtype=torch.int32, device="cuda")])
    params = torch.from_numpy(mbr.learned_params(lr_)).cuda()
    y = mbr.mlp_forward(params, q).cpu().numpy()[:n]
    b, lo, hi = _leaf_windows(y, info["n_leaves"], n)
    w = (hi[b] - lo[b] + 1).astype(np.float64)
    assert abs(w.mean() - info["mean_window"]) <= 1e-9 * info["mean_window"]
    lv_learned = np.ceil(np.log(np.maximum(w, 1)) / np.log(16))
    lv_whole = np.ceil(np.log(n) / np.log(16))
    saved = lv_whole - lv_learned.mean()
    say("chain: whole-list levels", lv_whole, "learned levels (mean)", lv_learned.mean(),
        "mean window", w.mean(), "of", n)
    assert w.mean() * 10 <= n
    assert saved >= 0.5
    # and the answers of both stay exact
    idx = torch.arange(n, dtype=torch.int32, device="cuda")
    assert torch.equal(mbr.rank_batch(lr_, st), idx)
    assert torch.equal(mbr.rank_batch(sampled, st), idx)
