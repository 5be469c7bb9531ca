"""Poisson on the square [-1,1]^2 with zero Dirichlet data: exact discrete
solution, Algorithm 2 written out, and the closed form of its J-th iterate.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper passages:
* (3.2): u = sum_ij X_ij (1-y^2)(1-x^2) C~_i(y) C~_j(x); rows <-> y.
* (3.6): M X D^T + D X M^T = F_C, the discrete system; F_C are the C~ x C~
  coefficients of f (Sec. 3.4).
* (3.8)-(3.9): with D = -S^2, S = diag(sqrt((j+1)(j+2))), the similarity
  transform turns A = D^-1 M into the symmetric A~ = -S^-1 M S^-1.  The
  unknown transforms by congruence: X = S^-1 Y S^-1, G = S^-1 F_C S^-1, so
  A~ Y - Y B~ = G with B~ = -A~ (the printed Y = D_s^-1 X D_s is read as
  Y = D_s^-1 X D_s^-1 with D_s = S^-1).
* App. B, proof of Lemma B.1: A~ decouples into its even- and odd-indexed
  principal submatrices, both tridiagonal.
* Algorithm 2: X_0 = 0; for j < J: solve X_{j+1/2}(B - p_j I) = F - (A - p_j I) X_j,
  then (A - q_j I) X_{j+1} = F - X_{j+1/2}(B - q_j I).
* Table 1, step 4: Chebyshev coefficients of u, an (n+2) x (n+2) array because
  u has degree n+1 in each variable.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import basis


def s_diag(n: int) -> np.ndarray:
    """S = |D|^(1/2)."""
    return np.sqrt(-basis.D_diag(n))


def atilde_dense(n: int) -> np.ndarray:
    """A~ = -S^-1 M S^-1 (symmetric pentadiagonal with zero +-1 diagonals)."""
    s = s_diag(n)
    return -basis.mult_M(n) / np.outer(s, s)


def atilde_eig(n: int):
    """Eigen-decomposition of A~ by parity blocks: returns (lam, V) with
    A~ = V diag(lam) V^T, V n x n orthogonal (block structure kept dense)."""
    A = atilde_dense(n)
    lam = np.empty(n)
    V = np.zeros((n, n))
    for par in (0, 1):
        idx = np.arange(par, n, 2)
        if idx.size == 0:
            continue
        blk = A[np.ix_(idx, idx)]
        d = np.diag(blk).copy()
        e = np.diag(blk, 1).copy()
        if idx.size == 1:
            w, v = d, np.ones((1, 1))
        else:
            w, v = sla.eigh_tridiagonal(d, e)
        lam[idx] = w
        V[np.ix_(idx, idx)] = v
    return lam, V


def _parity_solve(G: np.ndarray, lam: np.ndarray, V: np.ndarray, weight) -> np.ndarray:
    """Y with Yhat = weight(lam_a, lam_b) * (V^T G V), Y = V Yhat V^T, using
    contiguous parity blocks (V is block diagonal under the parity split)."""
    n = G.shape[0]
    Y = np.zeros_like(G)
    blocks = [np.arange(par, n, 2) for par in (0, 1)]
    for ia in blocks:
        if ia.size == 0:
            continue
        Va = np.ascontiguousarray(V[np.ix_(ia, ia)])
        for ib in blocks:
            if ib.size == 0:
                continue
            Vb = np.ascontiguousarray(V[np.ix_(ib, ib)])
            Gab = np.ascontiguousarray(G[np.ix_(ia, ib)])
            Ghat = Va.T @ Gab @ Vb
            Yhat = Ghat * weight(lam[ia][:, None], lam[ib][None, :])
            Y[np.ix_(ia, ib)] = Va @ Yhat @ Vb.T
    return Y


def solve_symmetric_sylvester(G: np.ndarray, eig=None) -> np.ndarray:
    """Exact Y with A~ Y + Y A~ = G (Bartels-Stewart for symmetric A~)."""
    lam, V = atilde_eig(G.shape[0]) if eig is None else eig
    return _parity_solve(G, lam, V, lambda la, lb: 1.0 / (la + lb))


def adi_exact_iterate(G: np.ndarray, p: np.ndarray, eig=None) -> np.ndarray:
    """Closed form of the J-th iterate of Algorithm 2 for A = A~, B = -A~,
    q_j = -p_j, F = G, X_0 = 0.  Each double step maps the error E to
    C E C with C = (A~ + p)^-1 (A~ - p), so E_J = -V[Yhat o r r^T]V^T with
    r(lam) = prod (lam - p_j)/(lam + p_j), and Y_J = V[Yhat o (1 - r r^T)]V^T."""
    lam, V = atilde_eig(G.shape[0]) if eig is None else eig

    def r(la):
        out = np.ones_like(la)
        for pj in p:
            out = out * ((la - pj) / (la + pj))
        return out

    return _parity_solve(G, lam, V, lambda la, lb: (1.0 - r(la) * r(lb)) / (la + lb))


def adi_dense(A, B, F, p, q):
    """Algorithm 2 with dense LAPACK solves (small n only)."""
    n = F.shape[0]
    I = np.eye(n)
    X = np.zeros_like(F)
    for pj, qj in zip(p, q):
        rhs = F - (A - pj * I) @ X
        # X_half (B - p I) = rhs  <=>  (B - p I)^T X_half^T = rhs^T
        Xh = np.linalg.solve((B - pj * I).T, rhs.T).T
        X = np.linalg.solve(A - qj * I, F - Xh @ (B - qj * I))
    return X


def kron_solve_generalized(F_C: np.ndarray) -> np.ndarray:
    """Brute-force solve of (3.6) as one n^2 x n^2 linear system.  With
    row-major vec, A X B^T <-> (A kron B) vec(X)."""
    n = F_C.shape[0]
    M = basis.mult_M(n)
    D = np.diag(basis.D_diag(n))
    L = np.kron(M, D) + np.kron(D, M)
    return np.linalg.solve(L, F_C.reshape(-1)).reshape(n, n)


def rhs_ct(F_T: np.ndarray) -> np.ndarray:
    """F_C = R F_T R^T: C~ x C~ coefficients of f from its Chebyshev ones."""
    R = basis.cheb_to_ct(F_T.shape[0])
    return R @ F_T @ R.T


def solve_native(F_C: np.ndarray, eig=None) -> np.ndarray:
    """X solving (3.6) exactly, via the symmetric form (3.9)."""
    s = s_diag(F_C.shape[0])
    G = F_C / np.outer(s, s)
    Y = solve_symmetric_sylvester(G, eig)
    return Y / np.outer(s, s)


def to_chebyshev(X: np.ndarray) -> np.ndarray:
    """U (n+2) x (n+2): Chebyshev coefficients of the expansion (3.2)."""
    P = basis.recombined_to_cheb(X.shape[0])
    return P @ X @ P.T


def poisson_square(F_T: np.ndarray, out: str = "cheb") -> np.ndarray:
    """Exact discrete solution for the Chebyshev right-hand side F_T
    (n x n, rows <-> y).  out='cheb' -> U (n+2)^2, out='native' -> X."""
    X = solve_native(rhs_ct(F_T))
    return to_chebyshev(X) if out == "cheb" else X


def poisson_square_adi(F_T: np.ndarray, p: np.ndarray, out: str = "cheb") -> np.ndarray:
    """The J-step ADI result (closed form) pushed through the same maps."""
    n = F_T.shape[0]
    s = s_diag(n)
    G = rhs_ct(F_T) / np.outer(s, s)
    X = adi_exact_iterate(G, p) / np.outer(s, s)
    return to_chebyshev(X) if out == "cheb" else X
