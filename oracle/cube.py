"""Poisson on the cube [-1,1]^3 with zero Dirichlet data: exact discrete
solution of the Kronecker system.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper passages:
* (5.2): (D_xx + D_yy + D_zz) vec X = vec F with Kronecker products of
  A = D^-1 M and the identity.  Applying the Laplacian identity (3.5) in
  three variables gives (M x M x D + M x D x M + D x M x M) vec X = vec F_C;
  dividing by D in each mode is what turns it into (5.2), so the right-hand
  side of (5.2) is read as (D^-1 x D^-1 x D^-1) vec F_C.
* Layout: X[i, j, k] multiplies (1-z^2)(1-y^2)(1-x^2) C~_i(z) C~_j(y) C~_k(x);
  F_T[i, j, k] multiplies T_i(z) T_j(y) T_k(x).
"""
from __future__ import annotations

import numpy as np

from . import basis
from .square import atilde_eig, s_diag


def mode_product(T: np.ndarray, A: np.ndarray, mode: int) -> np.ndarray:
    """Multiply tensor T by matrix A along ``mode`` (A acts on that index)."""
    return np.moveaxis(np.tensordot(A, T, axes=([1], [mode])), 0, mode)


def rhs_ct(F_T: np.ndarray) -> np.ndarray:
    R = basis.cheb_to_ct(F_T.shape[0])
    out = F_T
    for m in range(3):
        out = mode_product(out, R, m)
    return out


def solve_native(F_C: np.ndarray) -> np.ndarray:
    """Exact X of the cube system.  In symmetric variables X = (S^-1)^{x3} Y:
    (A~ x A~ x I + A~ x I x A~ + I x A~ x A~) Y = -(S^-1)^{x3} F_C, diagonal
    in the eigenbasis of A~ with entries la lb + la lc + lb lc."""
    n = F_C.shape[0]
    s = s_diag(n)
    sinv = 1.0 / s
    G = F_C * sinv[:, None, None] * sinv[None, :, None] * sinv[None, None, :]
    lam, V = atilde_eig(n)
    Gh = G
    for m in range(3):
        Gh = mode_product(Gh, V.T, m)
    la = lam[:, None, None]
    lb = lam[None, :, None]
    lc = lam[None, None, :]
    Yh = -Gh / (la * lb + la * lc + lb * lc)
    Y = Yh
    for m in range(3):
        Y = mode_product(Y, V, m)
    return Y * sinv[:, None, None] * sinv[None, :, None] * sinv[None, None, :]


def kron_solve(F_C: np.ndarray) -> np.ndarray:
    """Brute force: (M x M x D + M x D x M + D x M x M) vec X = vec F_C."""
    n = F_C.shape[0]
    M = basis.mult_M(n)
    D = np.diag(basis.D_diag(n))
    L = (np.kron(np.kron(M, M), D) + np.kron(np.kron(M, D), M)
         + np.kron(np.kron(D, M), M))
    return np.linalg.solve(L, F_C.reshape(-1)).reshape(n, n, n)


def to_chebyshev(X: np.ndarray) -> np.ndarray:
    P = basis.recombined_to_cheb(X.shape[0])
    out = X
    for m in range(3):
        out = mode_product(out, P, m)
    return out


def poisson_cube(F_T: np.ndarray, out: str = "cheb") -> np.ndarray:
    X = solve_native(rhs_ct(F_T))
    return to_chebyshev(X) if out == "cheb" else X
