"""GPU parity of the generic operator (tuples of Eq. H applied in gather form,
Eq. Talpha2) against the oracle's tuple apply, with staggered and trie ranks,
on particle-number sectors and on total-momentum sectors of the Hubbard ring
(Sec. V.C), plus the basis-change invariant: the momentum sectors together
hold the real-space spectrum."""
import math

import numpy as np
import pytest

from oracle import combinatorics as OC
from oracle import hamiltonian as OH
from oracle import operators as OP
import synth
from tests._util import say

pytestmark = pytest.mark.gpu
mbr = pytest.importorskip("paper_2203_04158_amd")
torch = pytest.importorskip("torch")
EPS64 = 2.0 ** -52


def _random_nconserving(M, seed, n_u):
    u = synth.uniform01(seed, M * M + 5 * n_u)
    t = (2 * u[: M * M] - 1).reshape(M, M)
    t = 0.5 * (t + t.T)
    t[np.abs(t) < 0.4] = 0.0
    r = u[M * M:].reshape(n_u, 5)
    cl = [(int(a * M), int(b * M), int(c * M), int(d * M), 4 * e - 2) for a, b, c, d, e in r]
    return t, cl


def _oracle_terms(M, t, cl):
    out = []
    for i in range(M):
        for j in range(M):
            if t[i, j] != 0.0:
                out.append(OP.scale(OP.mul(OP.creator(i), OP.annihilator(j)), -t[i, j]))
    for i, j, k, l, U in cl:
        out.append(OP.scale(OP.product(OP.creator(i), OP.creator(j), OP.annihilator(l),
                                       OP.annihilator(k)), 0.25 * U))
    return [x for x in out if x[0] != 0]


def _check(sec, ranker, states, M, t, cl, seed):
    op = mbr.operator_create(sec, ranker, mbr.terms_from_hamiltonian(M, t, cl))
    x = 2 * synth.uniform01(seed, states.size) - 1
    y = torch.empty(states.size, dtype=torch.float64, device="cuda")
    mbr.operator_apply(op, torch.from_numpy(x).cuda(), y)
    want, ab = OH.apply(states, _oracle_terms(M, t, cl), x, with_abssum=True)
    got = y.cpu().numpy()
    bad = np.abs(got - want) > 64 * EPS64 * ab + 1e-300
    assert not bad.any(), (np.nonzero(bad)[0][:5], got[bad][:5], want[bad][:5])


@pytest.mark.parametrize("M,N,kind,k", [(12, 5, "stag", 4), (12, 5, "trie", 4), (16, 8, "stag", 8),
                                        (16, 8, "trie", 8), (14, 0, "stag", 7), (9, 9, "trie", 3),
                                        (20, 3, "trie", 8)])
def test_operator_particle_number_sector(M, N, kind, k):
    cons = OC.constraints(M, N)
    st = OC.sector_enumerate(M, cons)
    sec = mbr.sector_build(M, cons)
    r = mbr.build_staggered_tables(M, N, k) if kind == "stag" else mbr.build_trie(sec, k)
    t, cl = _random_nconserving(M, M * 10 + N, 3 * M)
    _check(sec, r, st, M, t, cl, seed=M + N)


def test_operator_u64_sector_and_ras_trie():
    # 36 orbitals (64-bit patterns) with the staggered table
    M, N = 36, 3
    st = OC.sector_enumerate(M, OC.constraints(M, N))
    sec = mbr.sector_build(M, OC.constraints(M, N), width_bits=64)
    t, cl = _random_nconserving(M, 5, 40)
    _check(sec, mbr.build_staggered_tables(M, N, 9, width_bits=64), st, M, t, cl, seed=3)


def _ring_momentum(L, U, tt=1.0):
    """Eq. Hk (reading: U/L on the interaction): orbital k for spin down,
    L + k for spin up; eps_k = -2t cos(2 pi k / L)."""
    M = 2 * L
    t = np.zeros((M, M))
    for k in range(L):
        e = -2 * tt * math.cos(2 * math.pi * k / L)
        t[k, k] = t[L + k, L + k] = -e
    cl = []
    for k1 in range(L):
        for k2 in range(L):
            for k3 in range(L):
                k4 = (k1 + k2 - k3) % L
                # (U/L) c+_{k1 up} c+_{k2 dn} c_{k3 dn} c_{k4 up} = 1/4 U' c+_i c+_j c_l c_k
                cl.append((L + k1, k2, L + k4, k3, 4.0 * U / L))
    return M, t, cl


def _momentum_sector(L, nu, nd, K):
    M = 2 * L
    cons = OC.spin_constraints(L, nu, nd)
    w = [k for k in range(L)] * 2
    st = OC.sector_enumerate(M, cons)
    mom = np.array([sum(w[i] for i in range(M) if (int(a) >> i) & 1) % L for a in st])
    return cons, w, st[mom == K]


@pytest.mark.parametrize("L,nu,nd,K,k", [(6, 3, 3, 0, 4), (6, 3, 3, 2, 6), (8, 4, 4, 0, 8), (8, 3, 2, 5, 4)])
def test_operator_momentum_sector_trie(L, nu, nd, K, k):
    M, t, cl = _ring_momentum(L, 4.0)
    cons, w, st = _momentum_sector(L, nu, nd, K)
    sec = mbr.sector_build_mod(M, cons, w, L, K)
    assert sec.size == st.size
    assert np.array_equal(sec.states().cpu().numpy().view(np.uint32).astype(np.uint64), st)
    _check(sec, mbr.build_trie(sec, k), st, M, t, cl, seed=L + K)


def test_momentum_sectors_hold_the_real_space_spectrum():
    """Ring L = 6, (3,3), U = 4: the lowest eigenvalue over the six total-momentum
    sectors, from dense matrices of the GPU operator, equals the real-space E0."""
    L, nu, nd, U = 6, 3, 3, 4.0
    M, t, cl = _ring_momentum(L, U)
    terms = mbr.terms_from_hamiltonian(M, t, cl)
    lows, total = [], 0
    for K in range(L):
        cons, w, st = _momentum_sector(L, nu, nd, K)
        sec = mbr.sector_build_mod(M, cons, w, L, K)
        op = mbr.operator_create(sec, mbr.build_trie(sec, 6), terms)
        n = sec.size
        total += n
        H = np.zeros((n, n))
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        for j in range(n):
            e = torch.zeros(n, dtype=torch.float64, device="cuda")
            e[j] = 1.0
            mbr.operator_apply(op, e, y)
            H[:, j] = y.cpu().numpy()
        assert np.abs(H - H.T).max() <= 1e-12
        lows.append(np.linalg.eigvalsh(H)[0])
    assert total == math.comb(L, nu) * math.comb(L, nd)
    st = OH.sector(L, nu, nd)
    real = np.linalg.eigvalsh(OH.dense(st, OH.terms(L, OH.chain_bonds(L), U)))[0]
    say("momentum sector E0", lows, "real space", real)
    assert abs(min(lows) - real) <= 1e-10 * abs(real)
    assert abs(real - (-3.668706178873)) < 1e-9


def test_operator_rejects_bad_input():
    M, N = 10, 4
    sec = mbr.sector_build(M, OC.constraints(M, N))
    other = mbr.sector_build(M, OC.constraints(M, 5))
    terms = mbr.terms_from_hamiltonian(M, np.eye(M), [])
    with pytest.raises(mbr.MbrError):
        mbr.operator_create(sec, mbr.build_staggered_tables(M, 5, 4), terms)   # wrong C^M_N
    with pytest.raises(mbr.MbrError):
        mbr.operator_create(sec, mbr.build_trie(other, 4), terms)             # trie of another sector
    with pytest.raises(mbr.MbrError):
        mbr.operator_create(sec, mbr.build_trie(sec, 4), [(1.0, 1 << 12, 0, 0, 0, 0)])  # orbital >= M
    op = mbr.operator_create(sec, mbr.build_trie(sec, 4), terms)
    x = torch.zeros(sec.size, dtype=torch.float64, device="cuda")
    with pytest.raises(mbr.MbrError):
        mbr.operator_apply(op, x, x)                                          # aliasing


def test_operator_lanczos_momentum_and_particle_sectors():
    """E0 by the operator's GPU Lanczos: every total-momentum sector of the
    L = 6 ring against dense diagonalisation of the oracle's matrix, their
    minimum against the real-space E0, and a random Eq. H on C^12_5."""
    L, nu, nd, U = 6, 3, 3, 4.0
    M, t, cl = _ring_momentum(L, U)
    terms = mbr.terms_from_hamiltonian(M, t, cl)
    otl = _oracle_terms(M, t, cl)
    lows = []
    for K in range(L):
        cons, w, st = _momentum_sector(L, nu, nd, K)
        sec = mbr.sector_build_mod(M, cons, w, L, K)
        op = mbr.operator_create(sec, mbr.build_trie(sec, 6), terms)
        v0 = torch.from_numpy(synth.start_vector(K + 1, sec.size)).cuda()
        e0, nst, _, _ = mbr.operator_lanczos(op, v0, 120)
        want = np.linalg.eigvalsh(OH.dense(st, otl))[0]
        assert nst <= sec.size
        assert abs(e0 - want) <= 1e-9 * max(1.0, abs(want)), (K, e0, want, nst)
        lows.append(e0)
    assert abs(min(lows) - (-3.668706178873)) < 1e-9
    M, N = 12, 5
    st = OC.sector_enumerate(M, OC.constraints(M, N))
    sec = mbr.sector_build(M, OC.constraints(M, N))
    t, cl = _random_nconserving(M, 77, 30)
    cl = cl + [(k, l, i, j, U) for i, j, k, l, U in cl]   # add the Hermitian conjugates
    op = mbr.operator_create(sec, mbr.build_staggered_tables(M, N, 6), mbr.terms_from_hamiltonian(M, t, cl))
    e0, nst, a, b = mbr.operator_lanczos(op, torch.from_numpy(synth.start_vector(9, sec.size)).cuda(), 300)
    Hd = OH.dense(st, _oracle_terms(M, t, cl))
    assert np.abs(Hd - Hd.T).max() <= 1e-12
    want = np.linalg.eigvalsh(Hd)[0]
    assert abs(e0 - want) <= 1e-9 * max(1.0, abs(want)), (e0, want, nst)
    # the same run twice gives bitwise the same coefficients
    e1, nst1, a1, b1 = mbr.operator_lanczos(op, torch.from_numpy(synth.start_vector(9, sec.size)).cuda(), 300)
    assert e1 == e0 and nst1 == nst and np.array_equal(a[:nst], a1[:nst]) and np.array_equal(b[:nst], b1[:nst])
    # a sector smaller than the step count: the recurrence stops at its size
    # and the coefficients past the stop are zero
    sec = mbr.sector_build(6, OC.constraints(6, 2))
    op = mbr.operator_create(sec, mbr.build_staggered_tables(6, 2, 3),
                             mbr.terms_from_hamiltonian(6, np.eye(6) + 0.3 * np.ones((6, 6)), []))
    e2, n2, a2, b2 = mbr.operator_lanczos(op, torch.from_numpy(synth.start_vector(3, sec.size)).cuda(), 50)
    assert n2 <= sec.size and not a2[n2:].any() and not b2[n2 - 1:].any()
    st = OC.sector_enumerate(6, OC.constraints(6, 2))
    t6 = np.eye(6) + 0.3 * np.ones((6, 6))
    want = np.linalg.eigvalsh(OH.dense(st, _oracle_terms(6, t6, [])))[0]
    assert abs(e2 - want) <= 1e-10 * max(1.0, abs(want))


def test_operator_momentum_ring_l14_full_size_sampled():
    """The benchmark workload: L = 14, (7,7), total momentum 0 (841,332 states,
    2,772 tuples), k = 14 trie; sampled rows (first, last, and seeded) against
    the oracle's tuple apply, and an empty term list gives zero."""
    L, K = 14, 0
    M, t, cl = _ring_momentum(L, 4.0)
    cons = OC.spin_constraints(L, 7, 7)
    st = OH.sector(L, 7, 7)
    w = np.array([k for k in range(L)] * 2, dtype=np.int64)
    mom = np.zeros(st.size, dtype=np.int64)
    for i in range(M):
        mom += ((st >> np.uint64(i)) & np.uint64(1)).astype(np.int64) * w[i]
    st = st[mom % L == K]
    sec = mbr.sector_build_mod(M, cons, list(w), L, K)
    assert sec.size == st.size == 841332
    terms = mbr.terms_from_hamiltonian(M, t, cl)
    assert len(terms) == 2772
    op = mbr.operator_create(sec, mbr.build_trie(sec, 14), terms)
    x = 2 * synth.uniform01(21, st.size) - 1
    y = torch.empty(st.size, dtype=torch.float64, device="cuda")
    mbr.operator_apply(op, torch.from_numpy(x).cuda(), y)
    rows = np.unique(np.concatenate([[0, st.size - 1], synth.uniform_indices(22, 1500, st.size)]))
    want, ab = OH.apply(st, _oracle_terms(M, t, cl), x, rows=rows, with_abssum=True)
    got = y.cpu().numpy()[rows]
    assert (np.abs(got - want) <= 64 * EPS64 * ab + 1e-300).all()
    empty = mbr.operator_create(sec, mbr.build_trie(sec, 14), [])
    mbr.operator_apply(empty, torch.from_numpy(x).cuda(), y)
    assert not torch.any(y != 0)
