"""Hubbard-type Hamiltonians as lists of non-branching terms, applied on the fly.

Test infrastructure only (see the package docstring).  Conventions:
 * 2L spin-orbitals; spin-down orbital of site i is bit i, spin-up is bit L+i
   (spin-down in the least significant bits, as assumed for Eq. rankupdown);
 * H = - sum_bonds t_b sum_sigma (c+_{i sigma} c_{j sigma} + h.c.)
       + sum_i U_i c+_{i up} c+_{i dn} c_{i dn} c_{i up}
       + sum_{i sigma} eps_i n_{i sigma}
   (Eq. Hring generalised to an arbitrary bond list and on-site energies);
 * every term is built from the building blocks of Eqs. ci with the product
   rule of Appendix A and applied with Eq. Talpha2 (bra form), ranking the
   target by bisection.
"""
from __future__ import annotations

import numpy as np

from . import operators as ops
from ._clib import lib, ptr
from .combinatorics import sector_enumerate, spin_constraints


def chain_bonds(L: int, t: float = 1.0, periodic: bool = True):
    bonds = [(i, i + 1, t) for i in range(L - 1)]
    if periodic and L > 2:
        bonds.append((L - 1, 0, t))
    return bonds


def star_bonds(V):
    """Impurity (site 0) coupled to bath sites 1..n: hybridisation V_l enters
    H as +V_l (c+_0 c_l + h.c.), i.e. bond amplitude t = -V_l."""
    return [(0, l + 1, -float(v)) for l, v in enumerate(V)]


def terms(L: int, bonds, U, eps=None):
    """List of (v, m, l, r, x, s) tuples for H."""
    Ul = [float(U)] * L if np.isscalar(U) else [float(u) for u in U]
    out = []
    for (i, j, t) in bonds:
        for off in (0, L):
            a, b = i + off, j + off
            out.append(ops.scale(ops.mul(ops.creator(a), ops.annihilator(b)), -t))
            out.append(ops.scale(ops.mul(ops.creator(b), ops.annihilator(a)), -t))
    for i in range(L):
        if Ul[i] != 0.0:
            up, dn = L + i, i
            out.append(ops.scale(ops.product(ops.creator(up), ops.creator(dn),
                                             ops.annihilator(dn), ops.annihilator(up)), Ul[i]))
    if eps is not None:
        for i in range(L):
            if float(eps[i]) != 0.0:
                for off in (0, L):
                    out.append(ops.scale(ops.mul(ops.creator(i + off),
                                                 ops.annihilator(i + off)), float(eps[i])))
    return [t for t in out if t[0] != 0]


def apply_bisect(states, L: int, bonds, U, eps, x, row_range=None, threads: int = 1):
    """y = H x over rows row_range (default all) by the plain gather form with
    bisection ranks (the baseline method of Sec. V.B), on `threads` OpenMP
    threads.  Same Hamiltonian and conventions as terms()."""
    states = np.ascontiguousarray(states, dtype=np.uint64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    Ul = np.full(L, float(U)) if np.isscalar(U) else np.asarray(U, dtype=np.float64)
    el = np.zeros(L) if eps is None else np.asarray(eps, dtype=np.float64)
    bi = np.array([b[0] for b in bonds] or [0], dtype=np.int32)
    bj = np.array([b[1] for b in bonds] or [0], dtype=np.int32)
    bt = np.array([b[2] for b in bonds] or [0.0], dtype=np.float64)
    r0, r1 = row_range if row_range is not None else (0, states.size)
    y = np.empty(r1 - r0)
    rc = lib().orc_hubbard_bisect_apply(ptr(states), states.size, L, len(bonds), ptr(bi), ptr(bj), ptr(bt),
                                        ptr(np.ascontiguousarray(el)), ptr(np.ascontiguousarray(Ul)),
                                        ptr(x), ptr(y), r0, r1, threads)
    if rc != 0:
        raise ValueError(f"hop target of row {-rc - 1} is outside the sector")
    return y


def _arrays(tl):
    v = np.array([t[0] for t in tl], dtype=np.float64)
    f = [np.array([t[k] for t in tl], dtype=np.uint64) for k in (1, 2, 3, 4, 5)]
    return v, f[0], f[1], f[2], f[3], f[4]   # v, m, l, r, x, s


def sector(L: int, n_up: int, n_dn: int) -> np.ndarray:
    return sector_enumerate(2 * L, spin_constraints(L, n_up, n_dn))


def apply(states, tl, x, rows=None, with_abssum: bool = False, row_range=None):
    """y[rows] = (H x)[rows] by Eq. Talpha2 over the term list; row_range=(a, b)
    restricts the product to the contiguous rows a..b-1."""
    states = np.ascontiguousarray(states, dtype=np.uint64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    v, m, l, r, xx, s = _arrays(tl)
    L = lib()
    if rows is None:
        r0, r1 = row_range if row_range is not None else (0, states.size)
        y = np.empty(r1 - r0)
        a = np.empty(r1 - r0) if with_abssum else None
        rc = L.orc_apply_terms_bra(ptr(states), states.size, len(tl), ptr(v), ptr(m), ptr(l),
                                   ptr(xx), ptr(s), ptr(x), ptr(y),
                                   ptr(a) if a is not None else None, r0, r1)
        if rc != 0:
            raise ValueError(f"term leaves the sector at row {-rc - 1}")
        return (y, a) if with_abssum else y
    rows = np.asarray(rows, dtype=np.int64)
    y = np.empty(rows.size)
    a = np.empty(rows.size)
    one_y, one_a = np.empty(1), np.empty(1)
    for k, i in enumerate(rows):
        rc = L.orc_apply_terms_bra(ptr(states), states.size, len(tl), ptr(v), ptr(m), ptr(l),
                                   ptr(xx), ptr(s), ptr(x), ptr(one_y), ptr(one_a),
                                   int(i), int(i) + 1)
        if rc != 0:
            raise ValueError(f"term leaves the sector at row {i}")
        y[k], a[k] = one_y[0], one_a[0]
    return (y, a) if with_abssum else y


def sparse(states, tl):
    """The sector block of H as a scipy CSR matrix (entries from Eq. Talpha2)."""
    import scipy.sparse as sp
    states = np.ascontiguousarray(states, dtype=np.uint64)
    v, m, l, r, xx, s = _arrays(tl)
    L = lib()
    n = L.orc_terms_coo(ptr(states), states.size, len(tl), ptr(v), ptr(m), ptr(l), ptr(xx),
                        ptr(s), None, None, None, 0)
    if n < 0:
        raise ValueError(f"term leaves the sector at row {-n - 1}")
    rr = np.empty(n, dtype=np.int64)
    cc = np.empty(n, dtype=np.int64)
    vv = np.empty(n)
    L.orc_terms_coo(ptr(states), states.size, len(tl), ptr(v), ptr(m), ptr(l), ptr(xx), ptr(s),
                    ptr(rr), ptr(cc), ptr(vv), n)
    return sp.csr_matrix((vv, (rr, cc)), shape=(states.size, states.size))


def dense(states, tl) -> np.ndarray:
    return sparse(states, tl).toarray()


def dense_from_cee(L: int, bonds, U, eps=None) -> np.ndarray:
    """Full 2^(2L) matrix of H from products of the Eq. cee matrices
    (independent of the tuple algebra; tiny L only)."""
    M = 2 * L
    c = [ops.dense_annihilator(i, M) for i in range(M)]
    cd = [a.T for a in c]
    n = [cd[i] @ c[i] for i in range(M)]
    H = np.zeros((1 << M, 1 << M))
    Ul = [float(U)] * L if np.isscalar(U) else list(U)
    for (i, j, t) in bonds:
        for off in (0, L):
            H -= t * (cd[i + off] @ c[j + off] + cd[j + off] @ c[i + off])
    for i in range(L):
        H += Ul[i] * (cd[L + i] @ cd[i] @ c[i] @ c[L + i])
        if eps is not None:
            H += float(eps[i]) * (n[i] + n[L + i])
    return H


def one_body(L: int, bonds, eps=None) -> np.ndarray:
    """Single-particle matrix h with H_0 = sum_ij h_ij c+_i c_j per spin."""
    h = np.zeros((L, L))
    for (i, j, t) in bonds:
        h[i, j] -= t
        h[j, i] -= t
    if eps is not None:
        h[np.arange(L), np.arange(L)] += np.asarray(eps, dtype=np.float64)
    return h


def free_energy(L: int, bonds, n_up: int, n_dn: int, eps=None) -> float:
    """U = 0 ground energy: lowest n_up plus lowest n_dn single-particle levels."""
    e = np.linalg.eigvalsh(one_body(L, bonds, eps))
    return float(e[:n_up].sum() + e[:n_dn].sum())
