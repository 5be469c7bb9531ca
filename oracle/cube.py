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
* (5.3)-(5.9): the paper solves (5.2) by nested ADI: an outer iteration that
  splits D_zz from D_xx + D_yy, whose (x, y) half-step is itself an ADI
  iteration, whose slice solves are a third ADI.  ``kform_adi`` is a
  two-level form of the same nesting (derived here, not printed in the
  paper): with K = -A~^-1 (symmetric positive definite, spectrum in
  [1, 1/delta] by Lemma B.1) the symmetric cube system
  (A~ x A~ x I + A~ x I x A~ + I x A~ x A~) Y = -G becomes, after
  multiplying by (A~^-1)^{x3},
      (K_x + K_y + K_z) Y = B,   B = (A~^-1)^{x3} G,
  and every shifted solve (K + s I)^-1 = (s A~ - I)^-1 A~ is banded.  The
  outer ADI (Algorithm 2) splits H = K_x + K_y (spectrum in [2, 2/delta])
  from V = K_z (spectrum in [1, 1/delta]); its (x, y) half-step
  (H + q I) Y = R is, on every z-slice, the symmetric Sylvester equation
  (K + q/2) Y + Y (K + q/2) = R, solved by an inner Algorithm 2 to a tighter
  tolerance, as the paper's closing remark on the cube requires.
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


# --- two-level (K-form) nested ADI ----------------------------------------

def symmetric_rhs(F_C: np.ndarray) -> np.ndarray:
    """G = (S^-1)^{x3} F_C: the cube system in symmetric variables reads
    (A~ x A~ x I + A~ x I x A~ + I x A~ x A~) Y = -G with X = (S^-1)^{x3} Y."""
    n = F_C.shape[0]
    sinv = 1.0 / s_diag(n)
    return F_C * sinv[:, None, None] * sinv[None, :, None] * sinv[None, None, :]


def kform_rhs(G: np.ndarray) -> np.ndarray:
    """B = (A~^-1)^{x3} G (dense inverse; small n)."""
    from .square import atilde_dense
    Ai = np.linalg.inv(atilde_dense(G.shape[0]))
    B = G
    for m in range(3):
        B = mode_product(B, Ai, m)
    return B


def kform_outer_shifts(n: int, tol: float):
    """Algorithm 2 for (-H) Y - Y V = -B: sigma(-H) in [-2/delta, -2],
    sigma(V) in [1, 1/delta] (Lemma B.1 enclosure of A~ inverted)."""
    from .shifts import zolotarev_shifts
    delta = 1.0 / (30.0 * float(n) ** 4)
    return zolotarev_shifts(-2.0 / delta, -2.0, 1.0, 1.0 / delta, tol=tol)


def kform_inner_shifts(n: int, q: float, tol: float):
    """Algorithm 2 for -(K + q/2) Z - Z (K + q/2) = -R: symmetric intervals
    [-(1/delta + q/2), -(1 + q/2)] and [1 + q/2, 1/delta + q/2]."""
    from .shifts import zolotarev_shifts
    delta = 1.0 / (30.0 * float(n) ** 4)
    lo, hi = 1.0 + q / 2.0, 1.0 / delta + q / 2.0
    return zolotarev_shifts(-hi, -lo, lo, hi, tol=tol)


def _k_shift_solve(T: np.ndarray, s: float, mode: int, A: np.ndarray) -> np.ndarray:
    """(K + s I)^-1 along ``mode``, K = -A^-1: equals (s A - I)^-1 A."""
    n = A.shape[0]
    return mode_product(T, np.linalg.solve(s * A - np.eye(n), A), mode)


def _k_apply(T: np.ndarray, mode: int, Ainv: np.ndarray) -> np.ndarray:
    return mode_product(T, -Ainv, mode)


def kform_adi(G: np.ndarray, tol_outer: float, tol_inner: float, inner_exact: bool = False):
    """Y of the symmetric cube system by the two-level nested ADI (small n).

    Outer (Algorithm 2 with A = -H, B = V, F = -B):
        Y_{i+1/2} (V - p_i) = -B + (H + p_i) Y_i,
        (H + q_i) Y_{i+1}   =  B + (V - q_i) Y_{i+1/2},
    the second solved on each z-slice by an inner Algorithm 2 for
    A = -(K + q_i/2) (acting on y), B = K + q_i/2 (acting on x), F = -R, or
    exactly (eigendecomposition) when ``inner_exact``.
    Returns (Y, J_outer, [J_inner per outer step])."""
    from .square import atilde_dense, atilde_eig
    n = G.shape[0]
    A = atilde_dense(n)
    Ainv = np.linalg.inv(A)
    B = kform_rhs(G)
    J1, p1, q1 = kform_outer_shifts(n, tol_outer)
    lam, V = atilde_eig(n)
    kap = -1.0 / lam
    Y = np.zeros_like(B)
    inner_counts = []
    for pi, qi in zip(p1, q1):
        HY = _k_apply(Y, 1, Ainv) + _k_apply(Y, 2, Ainv)
        Yh = _k_shift_solve(-B + HY + pi * Y, -pi, 0, A)            # V acts on z (mode 0)
        R = B + _k_apply(Yh, 0, Ainv) - qi * Yh
        c = qi / 2.0
        if inner_exact:
            Rh = mode_product(mode_product(R, V.T, 1), V.T, 2)
            Zh = Rh / ((kap[None, :, None] + c) + (kap[None, None, :] + c))
            Y = mode_product(mode_product(Zh, V, 1), V, 2)
            inner_counts.append(0)
            continue
        J2, p2, q2 = kform_inner_shifts(n, qi, tol_inner)
        inner_counts.append(J2)
        Fi = -R
        Z = np.zeros_like(R)
        for pj, qj in zip(p2, q2):
            # Z_{1/2} (K + c - p_j) = F - (-(K + c) - p_j) Z, solved along x
            rhs = Fi + _k_apply(Z, 1, Ainv) + (c + pj) * Z
            Zh = _k_shift_solve(rhs, c - pj, 2, A)
            # -(K + c + q_j) Z = F - Z_{1/2} (K + c - q_j), solved along y
            rhs = Fi - (_k_apply(Zh, 2, Ainv) + (c - qj) * Zh)
            Z = -_k_shift_solve(rhs, c + qj, 1, A)
        Y = Z
    return Y, J1, inner_counts


def kform_outer_closed_form(G: np.ndarray, tol_outer: float) -> np.ndarray:
    """The J-th outer iterate with exact inner solves, in closed form: for
    commuting operators every eigen-triple (a, b, c) of (A~ x I x I, ...)
    evolves as in the scalar iteration, so
    Y_J = Y (1 - prod_j (a' - p_j)(b' - q_j) / ((a' - q_j)(b' - p_j))) with
    a' = -(k_y + k_x), b' = k_z eigenvalues of -H and V (k = -1/lambda)."""
    from .square import atilde_eig
    n = G.shape[0]
    lam, V = atilde_eig(n)
    kap = -1.0 / lam
    B = kform_rhs(G)
    J1, p1, q1 = kform_outer_shifts(n, tol_outer)
    Bh = B
    for m in range(3):
        Bh = mode_product(Bh, V.T, m)
    kz = kap[:, None, None]
    ky = kap[None, :, None]
    kx = kap[None, None, :]
    a = -(ky + kx)
    b = kz + 0.0 * a
    Ystar = Bh / (kx + ky + kz)
    r = np.ones_like(Ystar)
    for pj, qj in zip(p1, q1):
        r = r * ((a - pj) * (b - qj)) / ((a - qj) * (b - pj))
    Yh = Ystar * (1.0 - r)
    for m in range(3):
        Yh = mode_product(Yh, V, m)
    return Yh


# --- z-eigenbasis variant: one 2D ADI per z-slice ---------------------------

def zeig_slice_intervals(n: int, mu: float, lam_min: float, lam_max: float):
    """Intervals of Algorithm 2 for the slice equation in the z-eigenbasis.

    With P = A~ + mu I (mu an eigenvalue of A~), the slice equation
    P Y P - mu^2 Y = -G^ becomes, for Z = P Y,
        (-mu^2 P^-1) Z - Z (-P) = -G^,
    with sigma(-mu^2 P^-1) in [mu^2/(|lmin| + |mu|), mu^2/(|lmax| + |mu|)]
    and sigma(-P) in [|lmax| + |mu|, |lmin| + |mu|] for sigma(A~) in
    [lmin, lmax] (both negative): separated by |mu|."""
    m = abs(mu)
    return (mu * mu / (abs(lam_min) + m), mu * mu / (abs(lam_max) + m),
            abs(lam_max) + m, abs(lam_min) + m)


def zeig_adi(G: np.ndarray, tol: float, tight: bool = True):
    """Y of the symmetric cube system through the z-eigenbasis: transform G
    along z with the eigenvectors of A~, run Algorithm 2 on every slice
    (A = -mu^2 P^-1 on the left (y), B = -P on the right (x), F = -G^), then
    Y = P^-1 Z and transform back.  Dense small-n version.  Returns (Y, J per
    slice)."""
    from .shifts import square_enclosure, zolotarev_shifts
    from .square import atilde_dense, atilde_eig
    n = G.shape[0]
    A = atilde_dense(n)
    I = np.eye(n)
    lam, V = atilde_eig(n)
    if tight:
        lmin, lmax = lam.min() * (1 + 1e-6), lam.max() * (1 - 1e-6)
    else:
        lmin, lmax = square_enclosure(n)[0:2]
    Gh = mode_product(G, V.T, 0)
    Yh = np.empty_like(Gh)
    counts = []
    for c, mu in enumerate(lam):
        P = A + mu * I
        a, b, cc, d = zeig_slice_intervals(n, mu, lmin, lmax)
        J, p, q = zolotarev_shifts(a, b, cc, d, tol=tol)
        counts.append(J)
        As = -mu * mu * np.linalg.inv(P)
        Bs = -P
        F = -Gh[c]
        Z = np.zeros_like(F)
        for pj, qj in zip(p, q):
            Zh = np.linalg.solve((Bs - pj * I).T, (F - (As - pj * I) @ Z).T).T
            Z = np.linalg.solve(As - qj * I, F - Zh @ (Bs - qj * I))
        Yh[c] = np.linalg.solve(P, Z)
    return mode_product(Yh, V, 0), counts
