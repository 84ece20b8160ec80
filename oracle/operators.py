"""Non-branching terms (Appendix A) and the annihilator of Eq. cee.

Test infrastructure only (see the package docstring).  A term is the tuple
(v, m, l, r, x, s) of Eqs. Talpha1/Talpha2.
"""
from __future__ import annotations

import numpy as np


def _h(a: int) -> int:
    return bin(a).count("1")


def annihilator(i: int):
    """Eqs. ci: c_i has v = 1, m = r = x = 2^i, l = 0, s = 2^i - 1."""
    return (1, 1 << i, 0, 1 << i, 1 << i, (1 << i) - 1)


def creator(i: int):
    """c_i^dagger: the annihilator with l and r exchanged."""
    v, m, l, r, x, s = annihilator(i)
    return (v, m, r, l, x, s)


def scale(t, c):
    v, m, l, r, x, s = t
    return (v * c, m, l, r, x, s)


def _inside(m: int):
    """Every pattern whose set bits lie inside the mask m (0 and m included)."""
    sub = m
    while True:
        yield sub
        if sub == 0:
            return
        sub = (sub - 1) & m


def mul(ta, tb):
    """Tuple of the product T_a T_b (T_b acts first), Appendix A, read off from
    what the product does to states (Eq. Talpha1 applied twice).

    The product touches only the orbitals of m = m_a | m_b.  It is applied to
    every pattern inside m; for a product of non-branching terms at most one of
    them survives, and that one is r, with l = its image and x = l ^ r.  v is
    the coefficient on r itself (no orbital outside m occupied).  An orbital k
    outside m belongs to the sign mask s when occupying it flips the sign of
    the product.  No surviving pattern: the product vanishes (v = 0)."""
    m = ta[1] | tb[1]

    def act(alpha):
        c1, b1 = apply_ket(tb, alpha)
        if b1 is None:
            return 0, None
        c2, b2 = apply_ket(ta, b1)
        return (0, None) if b2 is None else (c1 * c2, b2)

    hits = [(beta,) + act(beta) for beta in _inside(m)]
    hits = [h for h in hits if h[2] is not None]
    if not hits:
        return (0, m, 0, 0, 0, 0)
    assert len(hits) == 1, "a product of non-branching terms is non-branching"
    r, v, img = hits[0]
    assert img & ~m == 0
    s = 0
    for k in range((m | ta[5] | tb[5]).bit_length()):
        if (m >> k) & 1:
            continue
        c, b = act(r | (1 << k))
        assert b == img | (1 << k) and abs(c) == abs(v)
        if c != v:
            s |= 1 << k
    return (v, m, img, r, img ^ r, s)


def product(*terms):
    out = terms[0]
    for t in terms[1:]:
        out = mul(out, t)
    return out


def apply_ket(t, alpha: int):
    """Eq. Talpha1: T|alpha> = v [alpha & m == r] (-1)^h(alpha & s) |alpha ^ x>.
    Returns (coefficient, pattern) or (0, None)."""
    v, m, l, r, x, s = t
    if v == 0 or (alpha & m) != r:
        return 0, None
    return (-v if _h(alpha & s) & 1 else v), alpha ^ x


def apply_bra(t, alpha: int):
    """Eq. Talpha2: <alpha|T = v [alpha & m == l] (-1)^h(alpha & s) <alpha ^ x|."""
    v, m, l, r, x, s = t
    if v == 0 or (alpha & m) != l:
        return 0, None
    return (-v if _h(alpha & s) & 1 else v), alpha ^ x


def dense_annihilator(i: int, M: int) -> np.ndarray:
    """Eq. cee as a 2^M x 2^M matrix: c_i|..n_i..> = [n_i = 1] prod_{j<i}(-1)^n_j |..0..>."""
    n = 1 << M
    c = np.zeros((n, n))
    for a in range(n):
        if (a >> i) & 1:
            c[a ^ (1 << i), a] = -1.0 if _h(a & ((1 << i) - 1)) & 1 else 1.0
    return c


def dense_of_term(t, M: int) -> np.ndarray:
    """Matrix of a term built column by column from Eq. Talpha1."""
    n = 1 << M
    T = np.zeros((n, n))
    for a in range(n):
        c, b = apply_ket(t, a)
        if b is not None:
            T[b, a] += c
    return T
