"""Poisson on the cylinder r <= 1, |z| <= 1 with zero Dirichlet data: exact
discrete solution of the paper's per-Fourier-mode systems (Sec. 4.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper passages and the readings taken:
* DFS doubling (4.2)-(4.3): r runs over [-1, 1]; f~(r, theta, z) =
  f(r cos theta, r sin theta, z) for every r (the doubled function), expanded
  in Chebyshev(r) x Fourier(theta) x Chebyshev(z) (4.4).  Mode k of f~ has the
  parity (-1)^k in r.
* Each mode solves (4.5); partial regularity (4.7) writes
  u~_k = r^m (1 - r^2)(1 - z^2) w_k with m = min(|k|, 2), and w_k is expanded
  in C~ x C~ ((4.9); C~ of Sec. 3.1).
* Case 1 (|k| >= 2): w satisfies (4.8),
    [L1 w - k^2 (1 - r^2) w](1 - z^2) + r^2 (1 - r^2) L2 w = f~_k,
  L1 w = r^2(1-r^2) w'' + (5 - 9r^2) r w' + 4(1 - 4r^2) w,
  L2 w = ((1 - z^2) w)_zz.  (Both checked by substituting u~_k into (4.5).)
  Reading: the matrices are the exact n x n Galerkin projections of these
  operators (test functions C~_i(r) C~_l(z), weight (1-r^2)(1-z^2)).  The
  printed matrix formula for L1 does not reproduce the zeroth-order term
  4(1 - 4r^2) of (4.8) (its identity and multiple of M give 8 - 16 r^2), and
  the printed A = (L1 - k^2 M)^-1 M omits the factor r^2 of the second term;
  the discrete system used here is
    P Y M + Q Y D = F_k,   P = [L1 - k^2 (1-r^2)],  Q = [r^2 (1-r^2)],
  with [op] the projection of op, M = [(1 - z^2)] and D of (3.6) in z.
* Case 2 (|k| = 1): P = [L3], L3 w = r(1-r^2) w'' + (3 - 7r^2) w' - 8 r w,
  Q = [r (1 - r^2)], right-hand side F_k.
* Case 3 (k = 0): P = [L4], L4 w = r^2(1-r^2) w'' + (1 - 5r^2) r w' - 4 r^2 w,
  Q = [r^2 (1 - r^2)], right-hand side [r^2] F_0 (the mode equation
  multiplied by r^2).
* Parity: w_k has the r-parity of k in Case 1 and is even in Cases 2 and 3;
  the equations are taken on the rows of the matching parity (Case 1 and 3:
  the same parity as w, Case 2: odd rows).  Components of F_k of the other
  parity are zero for doubled-up data and are ignored.
* Input: F (n_theta, n, n) complex, mode k = index - n_theta/2, rows <-> r
  Chebyshev, columns <-> z Chebyshev.  Output: U (n_theta, n + 4, n + 2)
  complex Chebyshev coefficients of u~_k (r-degree up to n + 3).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import basis
from .square import rhs_ct


def gegenbauer(n: int, lam: float, x: np.ndarray) -> np.ndarray:
    """C^(lam)_k(x), k = 0..n-1, shape (n, len(x)), by the three-term
    recurrence (k+1) C_{k+1} = 2(k+lam) x C_k - (k+2lam-1) C_{k-1}
    (NIST 18.9.1), C_0 = 1, C_1 = 2 lam x."""
    x = np.asarray(x, dtype=np.float64)
    C = np.zeros((max(n, 0), x.size))
    if n <= 0:
        return C
    C[0] = 1.0
    if n > 1:
        C[1] = 2 * lam * x
    for k in range(1, n - 1):
        C[k + 1] = (2 * (k + lam) * x * C[k] - (k + 2 * lam - 1) * C[k - 1]) / (k + 1)
    return C


def ct_and_derivatives(n: int, x: np.ndarray):
    """(C~_j, C~_j', C~_j'') at x for j < n: d/dx C^(l)_k = 2 l C^(l+1)_{k-1}
    (NIST 18.9.19), and C~_j = nu_j C^(3/2)_j (Sec. 3.1 footnote)."""
    j = np.arange(n, dtype=np.float64)
    nu = np.sqrt((j + 1.5) / ((j + 1) * (j + 2)))
    c0 = gegenbauer(n, 1.5, x) * nu[:, None]
    c1 = np.zeros_like(c0)
    c2 = np.zeros_like(c0)
    if n > 1:
        c1[1:] = 3.0 * gegenbauer(n - 1, 2.5, x) * nu[1:, None]
    if n > 2:
        c2[2:] = 15.0 * gegenbauer(n - 2, 3.5, x) * nu[2:, None]
    return c0, c1, c2


def galerkin(n: int, op) -> np.ndarray:
    """[op][i, j] = int C~_i(r) (op C~_j)(r) (1 - r^2) dr for i, j < n, with
    op(c0, c1, c2, r) returning the values of op applied to the basis
    (rows j) from the values of C~_j, C~_j', C~_j''.  Gauss-Jacobi quadrature
    with n + 4 nodes is exact (integrand degree <= 2n + 2)."""
    r, w = basis.gauss_jacobi11(n + 4)
    c0, c1, c2 = ct_and_derivatives(n, r)
    return (c0 * w[None, :]) @ op(c0, c1, c2, r).T


def mode_case(k: int) -> int:
    k = abs(k)
    return 1 if k >= 2 else (2 if k == 1 else 3)


def mode_operators(n: int, k: int):
    """(P, Q, rhs_map, m, w_parity, row_parity) of mode k."""
    case = mode_case(k)
    if case == 1:
        kk = float(k * k)
        P = galerkin(n, lambda c0, c1, c2, r: r * r * (1 - r * r) * c2 + (5 - 9 * r * r) * r * c1
                     + 4 * (1 - 4 * r * r) * c0 - kk * (1 - r * r) * c0)
        Q = galerkin(n, lambda c0, c1, c2, r: r * r * (1 - r * r) * c0)
        return P, Q, None, 2, abs(k) % 2, abs(k) % 2
    if case == 2:
        P = galerkin(n, lambda c0, c1, c2, r: r * (1 - r * r) * c2 + (3 - 7 * r * r) * c1 - 8 * r * c0)
        Q = galerkin(n, lambda c0, c1, c2, r: r * (1 - r * r) * c0)
        return P, Q, None, 1, 0, 1
    P = galerkin(n, lambda c0, c1, c2, r: r * r * (1 - r * r) * c2 + (1 - 5 * r * r) * r * c1
                 - 4 * r * r * c0)
    Q = galerkin(n, lambda c0, c1, c2, r: r * r * (1 - r * r) * c0)
    Mr2 = galerkin(n, lambda c0, c1, c2, r: r * r * c0)
    return P, Q, Mr2, 0, 0, 0


def z_operators(n: int):
    """M = [(1 - z^2)] (entries (3.7)) and the diagonal of D (3.6)."""
    return basis.mult_M(n), basis.D_diag(n)


def solve_mode_kron(P, Q, Mz, Dz, R):
    """Brute force: P Y Mz + Q Y diag(Dz) = R as one linear system
    (row-major vec: A Y B^T <-> kron(A, B) vec Y)."""
    p, m = R.shape
    L = np.kron(P, Mz.T) + np.kron(Q, np.diag(Dz))
    return np.linalg.solve(L, R.reshape(-1)).reshape(p, m)


def solve_mode_bs(P, Q, Mz, Dz, R):
    """Bartels-Stewart (scipy.linalg.solve_sylvester): with P invertible,
    (P^-1 Q) Y + Y (Mz D^-1) = P^-1 R D^-1."""
    Pinv_Q = np.linalg.solve(P, Q)
    rhs = np.linalg.solve(P, R) / Dz[None, :]
    return sla.solve_sylvester(Pinv_Q, Mz / Dz[None, :], rhs)


def r_output_map(n: int, m: int, N: int) -> np.ndarray:
    """Chebyshev coefficients (N rows) of r^m (1 - r^2) C~_i(r), i < n: those
    of (1 - r^2) C~_i (basis.recombined_to_cheb, exact entrywise) multiplied
    by r m times in coefficient space, x T_0 = T_1 and
    x T_k = (T_{k+1} + T_{k-1})/2 (degree i + m + 2 <= N - 1)."""
    if N < n + 2 + m:
        raise ValueError("N too small for r^m (1 - r^2) C~_i")
    P = np.zeros((N, n))
    P[:n + 2] = basis.recombined_to_cheb(n)
    for _ in range(m):
        Q = np.zeros_like(P)
        Q[1] += P[0]
        Q[2:] += P[1:-1] / 2
        Q[:-1] += P[1:] / 2
        P = Q
    return P


def solve_mode(F_T: np.ndarray, k: int, method: str = "bs") -> np.ndarray:
    """Chebyshev coefficients ((n+4) x (n+2), real) of u~_k for the real
    right-hand side F_T (n x n Chebyshev coefficients of one real part of
    f~_k)."""
    n = F_T.shape[0]
    P, Q, Mr2, m, wp, rp = mode_operators(n, k)
    Mz, Dz = z_operators(n)
    Fc = rhs_ct(F_T)
    if Mr2 is not None:
        Fc = Mr2 @ Fc
    wi = np.arange(wp, n, 2)
    ri = np.arange(rp, n, 2)
    Y = np.zeros((n, n))
    if wi.size and ri.size:
        Pp, Qp, Rp = P[np.ix_(ri, wi)], Q[np.ix_(ri, wi)], Fc[ri, :]
        solver = solve_mode_kron if method == "kron" else solve_mode_bs
        Y[wi, :] = solver(Pp, Qp, Mz, Dz, Rp)
    Pr = r_output_map(n, m, n + 4)
    Pz = basis.recombined_to_cheb(n)
    return Pr @ Y @ Pz.T


def poisson_cylinder(F: np.ndarray, method: str = "bs") -> np.ndarray:
    """U (n_theta, n+4, n+2) complex for the doubled-up right-hand side F
    (n_theta, n, n) complex (mode k = index - n_theta/2)."""
    nt, n, _ = F.shape
    U = np.zeros((nt, n + 4, n + 2), dtype=np.complex128)
    for idx in range(nt):
        k = idx - nt // 2
        U[idx] = (solve_mode(np.ascontiguousarray(F[idx].real), k, method)
                  + 1j * solve_mode(np.ascontiguousarray(F[idx].imag), k, method))
    return U


def evaluate(U: np.ndarray, r: np.ndarray, theta: np.ndarray, z: np.ndarray) -> np.ndarray:
    """u~(r, theta, z) = sum_k U_k(r, z) e^{i k theta} at matching points."""
    nt = U.shape[0]
    ks = np.arange(nt) - nt // 2
    Tr = basis.cheb_T(U.shape[1], r)
    Tz = basis.cheb_T(U.shape[2], z)
    vals = np.einsum("kij,im,jm->km", U, Tr, Tz)
    return np.einsum("km,km->m", vals, np.exp(1j * np.outer(ks, theta)))
