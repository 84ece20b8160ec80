"""Pins for oracle.hamiltonian and oracle.lanczos: dense Eq. cee construction,
closed forms, symmetries, and the tridiagonal solver."""
import math

import numpy as np
import pytest

from oracle import combinatorics as C
from oracle import hamiltonian as H
from oracle import lanczos as LZ
from synth import anderson_parameters, start_vector


def _sector_block(Hfull, states):
    idx = np.asarray(states, dtype=np.int64)
    return Hfull[np.ix_(idx, idx)]


@pytest.mark.parametrize("L,periodic", [(2, False), (3, True), (3, False), (4, True)])
def test_terms_match_dense_cee(L, periodic):
    bonds = H.chain_bonds(L, 0.7, periodic)
    U = [4.0, 1.5, 0.0, 2.0][:L]
    eps = [0.3, -0.2, 0.1, 0.05][:L]
    Hd = H.dense_from_cee(L, bonds, U, eps)
    full = np.arange(1 << (2 * L), dtype=np.uint64)
    assert np.abs(H.dense(full, H.terms(L, bonds, U, eps)) - Hd).max() < 1e-13
    # block diagonal in (N_up, N_dn): each sector block equals the restriction
    for nu in range(L + 1):
        for nd in range(L + 1):
            s = H.sector(L, nu, nd)
            Hs = H.dense(s, H.terms(L, bonds, U, eps))
            assert np.abs(Hs - _sector_block(Hd, s)).max() < 1e-13


def test_apply_matches_matrix():
    L = 5
    tl = H.terms(L, H.chain_bonds(L), 3.0)
    s = H.sector(L, 2, 3)
    x = start_vector(3, s.size)
    y = H.apply(s, tl, x)
    assert np.allclose(y, H.sparse(s, tl) @ x, atol=1e-14)
    rows = np.array([0, 7, s.size - 1])
    yr, ab = H.apply(s, tl, x, rows=rows, with_abssum=True)
    assert np.array_equal(yr, y[rows]) and (ab >= np.abs(yr)).all()


def test_open_dimer_closed_form():
    for U in (0.0, 1.0, 4.0, 10.0):
        s = H.sector(2, 1, 1)
        e = LZ.lowest_eigenvalue(H.dense(s, H.terms(2, [(0, 1, 1.0)], U)))
        assert abs(e - (U / 2 - math.sqrt(U * U / 4 + 4))) < 1e-12


@pytest.mark.parametrize("L,nu,nd", [(6, 3, 3), (8, 4, 4), (8, 3, 2), (10, 5, 5)])
def test_free_fermions(L, nu, nd):
    bonds = H.chain_bonds(L)
    s = H.sector(L, nu, nd)
    e = LZ.lowest_eigenvalue(H.sparse(s, H.terms(L, bonds, 0.0)))
    k = 2 * np.pi * np.arange(L) / L
    lev = np.sort(-2 * np.cos(k))
    assert abs(e - (lev[:nu].sum() + lev[:nd].sum())) < 1e-10
    assert abs(e - H.free_energy(L, bonds, nu, nd)) < 1e-10


def test_free_fermion_value_l14():
    # U = 0, L = 14 periodic, 7 + 7 particles: -4 t / sin(pi / 14)
    e = H.free_energy(14, H.chain_bonds(14), 7, 7)
    assert abs(e - (-4.0 / math.sin(math.pi / 14))) < 1e-12
    assert abs(e - (-17.975836829739738)) < 1e-12


def test_atomic_limit():
    L = 5
    for nu, nd in [(2, 3), (4, 3), (5, 5), (1, 1)]:
        s = H.sector(L, nu, nd)
        e = LZ.lowest_eigenvalue(H.dense(s, H.terms(L, H.chain_bonds(L, 0.0), 3.0)))
        assert abs(e - 3.0 * max(0, nu + nd - L)) < 1e-12


def test_particle_hole():
    L, U = 6, 4.0
    bonds = H.chain_bonds(L)
    for nu, nd in [(2, 2), (3, 2), (1, 4)]:
        e1 = LZ.lowest_eigenvalue(H.sparse(H.sector(L, nu, nd), H.terms(L, bonds, U)))
        e2 = LZ.lowest_eigenvalue(H.sparse(H.sector(L, L - nu, L - nd), H.terms(L, bonds, U)))
        assert abs(e2 - (e1 + U * (L - nu - nd))) < 1e-10


def test_small_ring_values():
    # independent check of the conventions by the Eq. cee matrices at L = 4
    L, U = 4, 4.0
    bonds = H.chain_bonds(L)
    Hd = H.dense_from_cee(L, bonds, U)
    s = H.sector(L, 2, 2)
    want = np.linalg.eigvalsh(_sector_block(Hd, s))[0]
    got = LZ.lowest_eigenvalue(H.sparse(s, H.terms(L, bonds, U)))
    assert abs(got - want) < 1e-12
    assert abs(got - (-2.102748483462)) < 1e-9


def test_anderson_noninteracting():
    eps_b, V = anderson_parameters(5, 4)
    L = 5
    eps = np.concatenate([[-1.0], eps_b])
    bonds = H.star_bonds(V)
    for nu, nd in [(2, 3), (0, 1), (5, 2), (3, 3)]:
        s = H.sector(L, nu, nd)
        e = LZ.lowest_eigenvalue(H.dense(s, H.terms(L, bonds, 0.0, eps)))
        assert abs(e - H.free_energy(L, bonds, nu, nd, eps)) < 1e-10
    # impurity U only on site 0 vs the Eq. cee matrices
    U = [2.5, 0, 0, 0, 0]
    Hd = H.dense_from_cee(L, bonds, U, eps)
    s = H.sector(L, 2, 2)
    assert np.abs(H.dense(s, H.terms(L, bonds, U, eps)) - _sector_block(Hd, s)).max() < 1e-13


def test_tridiagonal_closed_form():
    for n in (1, 2, 5, 40, 200):
        e = LZ.tridiag_lowest(np.zeros(n), np.ones(n))
        assert abs(e - 2 * math.cos(math.pi * n / (n + 1))) < 1e-12


def test_lanczos_converges_to_lowest():
    L = 6
    s = H.sector(L, 3, 3)
    A = H.sparse(s, H.terms(L, H.chain_bonds(L), 4.0))
    want = np.linalg.eigvalsh(A.toarray())[0]
    assert abs(want - (-3.668706178873)) < 1e-9
    v0 = start_vector(2, s.size)
    a, b = LZ.lanczos(lambda v: A @ v, v0, 120)
    assert abs(LZ.tridiag_lowest(a, b) - want) < 1e-10
    a, b = LZ.lanczos(lambda v: A @ v, v0, s.size + 5, reorth=True, breakdown=1e-10)
    assert a.size <= s.size
    assert abs(LZ.tridiag_lowest(a, b) - want) < 1e-10


@pytest.mark.parametrize("L,periodic", [(2, False), (3, True), (4, True), (6, True)])
def test_bisect_gather_apply_matches_dense_cee(L, periodic):
    """The plain bisection gather form (the timed baseline) against the dense
    Eq. cee Hamiltonian at L <= 4 and against the tuple-built apply above."""
    bonds = H.chain_bonds(L, 0.7, periodic) + ([(0, L - 1, -0.3)] if L > 3 else [])
    U = list(np.linspace(4.0, 1.0, L))
    eps = list(np.linspace(-0.3, 0.2, L))
    Hd = H.dense_from_cee(L, bonds, U, eps) if L <= 4 else None
    tl = H.terms(L, bonds, U, eps)
    for nu in range(L + 1):
        for nd in range(L + 1):
            s = H.sector(L, nu, nd)
            x = start_vector(nu * 13 + nd + 1, s.size)
            y = H.apply_bisect(s, L, bonds, U, eps, x)
            want, ab = H.apply(s, tl, x, with_abssum=True)
            assert (np.abs(y - want) <= 64 * 2.0 ** -52 * ab + 1e-300).all()
            if Hd is not None:
                assert np.abs(y - _sector_block(Hd, s) @ x).max() < 1e-12


def test_bisect_gather_apply_impurity_threads_and_rows():
    eps_b, V = anderson_parameters(5, 5)
    L = 6
    eps = [-4.0] + list(eps_b)
    U = [8.0] + [0.0] * 5
    bonds = H.star_bonds(V)
    tl = H.terms(L, bonds, U, eps)
    s = H.sector(L, 3, 2)
    x = start_vector(9, s.size)
    y1 = H.apply_bisect(s, L, bonds, U, eps, x)
    y4 = H.apply_bisect(s, L, bonds, U, eps, x, threads=4)
    part = H.apply_bisect(s, L, bonds, U, eps, x, row_range=(17, 101), threads=3)
    want, ab = H.apply(s, tl, x, with_abssum=True)
    assert np.array_equal(y1, y4) and np.array_equal(part, y1[17:101])
    assert (np.abs(y1 - want) <= 64 * 2.0 ** -52 * ab + 1e-300).all()


def test_threaded_rank_batches_match():
    st = C.sector_enumerate(16, C.constraints(16, 7))
    q = np.concatenate([st[::3], np.arange(0, 1 << 17, 97, dtype=np.uint64)])
    b = C.rank_batch_threads(st, q, "bisect", 4)
    assert np.array_equal(b, C.bisect_rank(st, q))
    m = st[::5]
    assert np.array_equal(C.rank_batch_threads(st, m, "cns", 3), C.cns_rank_batch(m).astype(np.int64))
