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


def mul(ta, tb):
    """Product rule figure of Appendix A: tuple of T_a T_b from those of T_a, T_b."""
    va, ma, la, ra, xa, sa = ta
    vb, mb, lb, rb, xb, sb = tb
    # Pauli check on the intermediate state where both masks overlap.
    v = 0 if ((ra ^ lb) & ma & mb) else va * vb
    m = ma | mb
    r = rb | (ra & ~mb)
    l = la | (lb & ~ma)
    x = l ^ r
    s = (sa ^ sb) & ~m
    # Sign of T_a T_b on the state |r>, absorbed into v.
    z = r
    p = z & sb
    z ^= xb
    p ^= z & sa
    if _h(p) & 1:
        v = -v
    return (v, m, l, r, x, s)


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
