"""Pins for oracle.operators: Appendix A tuples against dense Eq. cee matrices."""
import numpy as np

from oracle import operators as O
from synth import splitmix64


def test_building_blocks_match_cee():
    M = 4
    for i in range(M):
        assert np.array_equal(O.dense_of_term(O.annihilator(i), M), O.dense_annihilator(i, M))
        assert np.array_equal(O.dense_of_term(O.creator(i), M), O.dense_annihilator(i, M).T)


def test_anticommutation_of_cee():
    M = 3
    c = [O.dense_annihilator(i, M) for i in range(M)]
    I = np.eye(1 << M)
    for i in range(M):
        for j in range(M):
            assert np.allclose(c[i] @ c[j].T + c[j].T @ c[i], I * (i == j))
            assert np.allclose(c[i] @ c[j] + c[j] @ c[i], 0)


def test_random_products_match_dense():
    M = 4
    dense = {}
    for i in range(M):
        dense[("c", i)] = O.dense_annihilator(i, M)
        dense[("d", i)] = O.dense_annihilator(i, M).T
    r = splitmix64(11, 4 * 3000)
    for k in range(3000):
        n = 1 + int(r[4 * k] % np.uint64(4))
        facs = []
        for f in range(n):
            code = int(r[4 * k + f] >> np.uint64(7)) % (2 * M)
            facs.append(("c" if code < M else "d", code % M))
        tl = [O.annihilator(i) if kind == "c" else O.creator(i) for kind, i in facs]
        T = O.product(*tl)
        D = np.eye(1 << M)
        for f in facs:
            D = D @ dense[f]
        assert np.array_equal(O.dense_of_term(T, M), D), facs
        # bra form is the transpose action
        for a in range(1 << M):
            c, b = O.apply_bra(T, a)
            row = D[a]
            if b is None:
                assert not row.any()
            else:
                assert row[b] == c and np.count_nonzero(row) == 1


def test_hop_sign_is_parity_between():
    # <alpha| c+_p c_q is non-zero iff alpha_p = 1, alpha_q = 0; its sign is the
    # parity of the occupied orbitals strictly between p and q.
    M = 6
    for p in range(M):
        for q in range(M):
            if p == q:
                continue
            T = O.mul(O.creator(p), O.annihilator(q))
            lo, hi = min(p, q), max(p, q)
            between = ((1 << hi) - 1) & ~((1 << (lo + 1)) - 1)
            for a in range(1 << M):
                c, b = O.apply_bra(T, a)
                if (a >> p) & 1 and not (a >> q) & 1:
                    assert b == a ^ (1 << p) ^ (1 << q)
                    assert c == (-1 if bin(a & between).count("1") & 1 else 1)
                else:
                    assert b is None
