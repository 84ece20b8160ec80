"""Lanczos ground-state search and tridiagonal eigenvalues (fp64).

Test infrastructure only (see the package docstring).  The paper uses the
Lanczos method for the lowest eigenvalue in a sector (Sec. I-II, Sec. V.B) but
does not spell it out; this is the textbook three-term recurrence
    u = H v_j - beta_{j-1} v_{j-1};  alpha_j = <v_j, u>;  w = u - alpha_j v_j;
    (optional full classical Gram-Schmidt of w against v_1..v_j);
    beta_j = |w|;  v_{j+1} = w / beta_j,
stopping early when beta_j <= breakdown.
"""
from __future__ import annotations

import numpy as np


def lanczos(matvec, v0, m: int, reorth: bool = False, breakdown: float = 0.0):
    """Returns (alpha[0..k-1], beta[0..k-1]); beta[j] couples steps j and j+1,
    and a breakdown at step k-1 leaves beta[k-1] = 0."""
    v = np.asarray(v0, dtype=np.float64).copy()
    v /= np.sqrt(np.dot(v, v))
    v_prev = np.zeros_like(v)
    b_prev = 0.0
    basis = [v.copy()] if reorth else None
    alphas, betas = [], []
    for _ in range(m):
        u = matvec(v) - b_prev * v_prev
        a = float(np.dot(v, u))
        w = u - a * v
        if reorth:
            Q = np.array(basis)
            w = w - Q.T @ (Q @ w)
        b = float(np.sqrt(np.dot(w, w)))
        alphas.append(a)
        if b <= breakdown:
            betas.append(0.0)
            break
        betas.append(b)
        v_prev, v, b_prev = v, w / b, b
        if reorth:
            basis.append(v.copy())
    return np.array(alphas), np.array(betas)


def tridiag_lowest(alpha, beta) -> float:
    """Lowest eigenvalue of the symmetric tridiagonal matrix with diagonal alpha
    and off-diagonal beta[:len(alpha)-1] (LAPACK via scipy)."""
    from scipy.linalg import eigh_tridiagonal
    alpha = np.asarray(alpha, dtype=np.float64)
    if alpha.size == 1:
        return float(alpha[0])
    off = np.asarray(beta, dtype=np.float64)[: alpha.size - 1]
    return float(eigh_tridiagonal(alpha, off, eigvals_only=True,
                                  select="i", select_range=(0, 0))[0])


def lowest_eigenvalue(H) -> float:
    """Lowest eigenvalue of a dense or sparse symmetric matrix (LAPACK/ARPACK)."""
    import scipy.sparse as sp
    if sp.issparse(H):
        if H.shape[0] <= 4000:
            return float(np.linalg.eigvalsh(H.toarray())[0])
        from scipy.sparse.linalg import eigsh
        return float(eigsh(H, k=1, which="SA", tol=1e-14, ncv=40,
                           v0=np.ones(H.shape[0]))[0][0])
    return float(np.linalg.eigvalsh(H)[0])
