"""Poisson on a rectangle [a,b] x [c,d] with Dirichlet data: exact discrete
solution.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper passages:
* The rectangle remark after Table 1: with s = (2x - a - b)/(b - a) and
  t = (2y - c - d)/(d - c), u_xx = sx^2 u_ss and u_yy = sy^2 u_tt with
  sx = 2/(b - a), sy = 2/(d - c); the discrete system (3.6) becomes
  sx^2 M X D + sy^2 D X M = F_C (rows <-> y as in (3.2)), and the
  symmetric form (3.9) sx^2 A~ Y + sy^2 Y A~ = G.  The two sides now carry
  different spectra, so Theorem 2.1 is used with general intervals.
* Sec. 6.1: nonhomogeneous Dirichlet data.  A function u_bc taking the
  boundary values is subtracted: solve Lap u0 = f - Lap u_bc with zero data,
  then u = u0 + u_bc, all in coefficient space.  Here u_bc is the
  transfinite (Coons) interpolant of the four boundary traces.
* Boundary data: four Chebyshev series of length n + 2 in the mapped
  variable: left u(a, y) and right u(b, y) in t, bottom u(x, c) and top
  u(x, d) in s; they must agree at the corners.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import chebyshev as npc

from . import basis, shifts
from .square import _parity_solve, atilde_dense, atilde_eig, rhs_ct, s_diag, to_chebyshev


def scalings(box):
    a, b, c, d = box
    return (2.0 / (b - a)) ** 2, (2.0 / (d - c)) ** 2


def solve_native_rect(F_C: np.ndarray, box) -> np.ndarray:
    """X of sx^2 M X D + sy^2 D X M = F_C (exact, eigen-decomposition)."""
    sx2, sy2 = scalings(box)
    n = F_C.shape[0]
    s = s_diag(n)
    G = F_C / np.outer(s, s)
    lam, V = atilde_eig(n)
    Y = _parity_solve(G, lam, V, lambda la, lb: 1.0 / (sx2 * la + sy2 * lb))
    return Y / np.outer(s, s)


def kron_solve_rect(F_C: np.ndarray, box) -> np.ndarray:
    """Brute-force solve of sx^2 M X D + sy^2 D X M = F_C as one n^2 x n^2
    system (row-major vec: A X B^T <-> kron(A, B) vec X)."""
    sx2, sy2 = scalings(box)
    n = F_C.shape[0]
    M = basis.mult_M(n)
    D = np.diag(basis.D_diag(n))
    L = sx2 * np.kron(M, D) + sy2 * np.kron(D, M)
    return np.linalg.solve(L, F_C.reshape(-1)).reshape(n, n)


def rect_enclosure(n: int, box, lam=None):
    """Intervals of Theorem 2.1 for A Y - Y B = G with A = sx^2 A~ (acting on
    rows) and B = -sy^2 A~ (columns): sigma(A~) in [lo, hi] (Lemma B.1's
    [-1, -1/(30 n^4)] unless given) scaled by sx^2, and the mirror image
    scaled by sy^2."""
    sx2, sy2 = scalings(box)
    lo, hi = (-1.0, -1.0 / (30.0 * n ** 4)) if lam is None else lam
    return sx2 * lo, sx2 * hi, -sy2 * hi, -sy2 * lo


def rect_shifts(n: int, box, tol: float, lam=None):
    return shifts.zolotarev_shifts(*rect_enclosure(n, box, lam), tol=tol)


def adi_iterate_rect(G: np.ndarray, box, p: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Closed form of the J-th iterate of Algorithm 2 (X_0 = 0) for
    A Y - Y B = G, A = sx^2 A~, B = -sy^2 A~.  Each step maps the error E to
    (A - q)^-1 (A - p) E (B - p)^-1 (B - q), so E_J = r(A) E_0 r(B)^-1 with
    r(z) = prod (z - p_j)/(z - q_j), and in the eigenbasis of A~
    Yhat_J = Yhat (1 - r(alpha_a) / r(beta_b)), alpha = sx^2 lam,
    beta = -sy^2 lam."""
    sx2, sy2 = scalings(box)
    lam, V = atilde_eig(G.shape[0])

    def r(z):
        out = np.ones_like(z)
        for pj, qj in zip(p, q):
            out = out * ((z - pj) / (z - qj))
        return out

    return _parity_solve(
        G, lam, V,
        lambda la, lb: (1.0 - r(sx2 * la) / r(-sy2 * lb)) / (sx2 * la + sy2 * lb))


def rect_operators(n: int, box):
    """Dense A = sx^2 A~ and B = -sy^2 A~ (small n; for Algorithm 2 with
    dense solves)."""
    sx2, sy2 = scalings(box)
    A = atilde_dense(n)
    return sx2 * A, -sy2 * A


def poisson_rect(F_T: np.ndarray, box, out: str = "cheb") -> np.ndarray:
    X = solve_native_rect(rhs_ct(F_T), box)
    return to_chebyshev(X) if out == "cheb" else X


def coons_coeffs(bc) -> np.ndarray:
    """Chebyshev coefficients (N x N, N = len of each trace, rows <-> t) of
    the transfinite interpolant
      u_bc = (1-s)/2 L(t) + (1+s)/2 R(t) + (1-t)/2 B(s) + (1+t)/2 T(s)
             - bilinear interpolant of the corner values B(-1), B(1), T(-1), T(1),
    term by term: a product f(t) g(s) of Chebyshev series has the outer
    product of their coefficient vectors as its 2-D coefficients, and
    (1 -+ s)/2 = T_0/2 -+ T_1/2.  (Exact zeros off rows 0, 1 and columns 0, 1:
    the lift's Laplacian multiplies coefficient k by up to k^4, so a sampled
    construction's rounding there would be amplified.)"""
    L, R, B, T = (np.asarray(v, dtype=np.float64) for v in bc)
    N = len(L)
    hm = np.zeros(N)
    hp = np.zeros(N)
    hm[0], hp[0] = 0.5, 0.5
    if N > 1:
        hm[1], hp[1] = -0.5, 0.5
    c00, c10 = npc.chebval(-1.0, B), npc.chebval(1.0, B)  # (s, t) = (-1, -1), (1, -1)
    c01, c11 = npc.chebval(-1.0, T), npc.chebval(1.0, T)  # (-1, 1), (1, 1)
    return (np.outer(L, hm) + np.outer(R, hp) + np.outer(hm, B) + np.outer(hp, T)
            - (c00 * np.outer(hm, hm) + c10 * np.outer(hm, hp) + c01 * np.outer(hp, hm)
               + c11 * np.outer(hp, hp)))


def coons_coeffs_sampled(bc) -> np.ndarray:
    """The same interpolant by sampling on the first-kind grid of size
    Ns x Ns, Ns = max(2, leading trace coefficients up to the last nonzero
    one), and the discrete cosine map (exact in exact arithmetic: u_bc has
    degree <= Ns - 1 in each variable).  Independent check of coons_coeffs."""
    L, R, B, T = (np.asarray(v, dtype=np.float64) for v in bc)
    N = len(L)
    nz = [np.nonzero(v)[0] for v in (L, R, B, T)]
    Ns = max([2] + [int(z[-1]) + 1 for z in nz if z.size])
    L, R, B, T = L[:Ns], R[:Ns], B[:Ns], T[:Ns]
    x = basis.cheb_points(Ns)
    S, Tt = np.meshgrid(x, x, indexing="xy")  # S varies along columns (s), Tt along rows (t)
    Lv, Rv = npc.chebval(Tt, L), npc.chebval(Tt, R)
    Bv, Tv = npc.chebval(S, B), npc.chebval(S, T)
    c00, c10 = npc.chebval(-1.0, B), npc.chebval(1.0, B)
    c01, c11 = npc.chebval(-1.0, T), npc.chebval(1.0, T)
    vals = ((1 - S) / 2 * Lv + (1 + S) / 2 * Rv + (1 - Tt) / 2 * Bv + (1 + Tt) / 2 * Tv
            - ((1 - S) * (1 - Tt) * c00 + (1 + S) * (1 - Tt) * c10
               + (1 - S) * (1 + Tt) * c01 + (1 + S) * (1 + Tt) * c11) / 4)
    D = basis.dct_matrix(Ns)
    out = np.zeros((N, N))
    out[:Ns, :Ns] = D @ vals @ D.T
    return out


def laplacian_coeffs(U: np.ndarray, box) -> np.ndarray:
    """Chebyshev coefficients (same shape as U, rows <-> t) of
    sx^2 u_ss + sy^2 u_tt for u with coefficients U (library
    differentiation of the coefficient array along each axis)."""
    sx2, sy2 = scalings(box)
    out = np.zeros_like(U, dtype=np.float64)
    Uss = npc.chebder(U, m=2, axis=1)
    Utt = npc.chebder(U, m=2, axis=0)
    out[:, : Uss.shape[1]] += sx2 * Uss
    out[: Utt.shape[0], :] += sy2 * Utt
    return out


def cheb_to_ct_rect(n: int, N: int) -> np.ndarray:
    """R (n x N), R[i, k] = int T_k C~_i (1 - x^2) dx: the first n C~
    coefficients of T_k for k < N (footnote of Sec. 3.1), by Gauss-Jacobi
    quadrature with n + N nodes (exact for the degree n + N - 2 integrand)."""
    x, w = basis.gauss_jacobi11(n + N)
    return (basis.ct_values(n, x) * w[None, :]) @ basis.cheb_T(N, x).T


def cheb_to_ct_closed(n: int, N: int, dtype=np.float64) -> np.ndarray:
    """R (n x N) with R[i, k] = C~_i coefficient of T_k, entrywise to
    relative accuracy, from the Gegenbauer connection formula (DLMF 18.18.16)
    in the limit lambda -> 0 that gives T_k (DLMF 18.7.25):
      T_k = (k/2) sum_l (k-l-1)! (-mu)_l (k - 2l + mu) / ((mu)_{k-l+1} l!) C^(mu)_{k-2l},
    mu = 3/2, and C^(3/2)_i = C~_i / nu_i with nu_i = sqrt((i+3/2)/((i+1)(i+2)))
    (footnote of Sec. 3.1).  The factors are accumulated as products of
    ratios (relative error ~ k eps), unlike the quadrature of cheb_to_ct_rect
    whose absolute error ~ eps swamps the small far-from-diagonal entries
    when they multiply large coefficients.  dtype=np.longdouble evaluates in
    extended precision."""
    mu = dtype(1.5)
    R = np.zeros((n, N), dtype=dtype)
    if n == 0 or N == 0:
        return R
    i_all = np.arange(n, dtype=dtype)
    nu = np.sqrt((i_all + dtype(1.5)) / ((i_all + 1) * (i_all + 2)))
    R[0, 0] = 1 / nu[0]  # T_0 = C^(mu)_0
    k = np.arange(1, N, dtype=dtype)
    # t_0(k) = (k-1)! / (mu)_{k+1}, by t_0(1) = 1/(mu (mu+1)) and
    # t_0(k) / t_0(k-1) = (k-1) / (mu + k)
    t = np.cumprod(np.concatenate([np.array([1 / (mu * (mu + 1))], dtype=dtype),
                                   (k[1:] - 1) / (mu + k[1:])]))
    for l in range((N - 1) // 2 + 1):
        i = k - 2 * l
        ok = (i >= 0) & (i < n)
        ii = i[ok].astype(int)
        R[ii, k[ok].astype(int)] = (k[ok] / 2) * t[ok] * (i[ok] + mu) / nu[ii]
        # t_{l+1} / t_l = (mu + k - l) (l - mu) / ((k - l - 1) (l + 1)); columns
        # whose last term has passed are never read again
        with np.errstate(divide="ignore", invalid="ignore"):
            t = t * (mu + k - l) * (l - mu) / ((k - l - 1) * (l + 1))
    return R


def ct_projection(C_T: np.ndarray, n: int) -> np.ndarray:
    """First n x n C~ x C~ coefficients of a function given by a Chebyshev
    coefficient array of any size (the closed-form map on both axes)."""
    Ra = cheb_to_ct_closed(n, C_T.shape[0])
    Rb = Ra if C_T.shape[1] == C_T.shape[0] else cheb_to_ct_closed(n, C_T.shape[1])
    return Ra @ C_T @ Rb.T


def cheb_second_derivative(c: np.ndarray) -> np.ndarray:
    """Chebyshev coefficients of g'' for g = sum c_k T_k, by the derivative
    recurrence d_{k-1} = d_{k+1} + 2 k c_k (d_0 halved) applied twice, in the
    dtype of c."""
    def der(c):
        N = len(c)
        d = np.zeros(max(N - 1, 0), dtype=c.dtype)
        for k in range(N - 1, 0, -1):
            d[k - 1] = (d[k + 1] if k + 1 < N - 1 else 0) + 2 * k * c[k]
        if N > 1:
            d[0] = d[0] / 2
        return d
    return der(der(np.asarray(c)))


def lift_correction(bc, box, n: int) -> np.ndarray:
    """C~ x C~ coefficients (n x n) of Lap u_bc for the transfinite lift:
    differentiating each product term of u_bc,
      Lap u_bc = sx2 [(1-t)/2 B''(s) + (1+t)/2 T''(s)] + sy2 [(1-s)/2 L''(t) + (1+s)/2 R''(t)],
    so the 2-D projection is a sum of outer products of 1-D C~ coefficient
    vectors.  The 1-D projections C~(g'') are evaluated in extended precision
    (np.longdouble): for rough traces the sum R g'' cancels by up to ~4e3
    (moduli over result at n = 1024-4096, coefficients ~ k^-2), which in
    float64 leaves ~1e-11 relative error in U."""
    ld = np.longdouble
    sx2, sy2 = scalings(box)
    R = cheb_to_ct_closed(n, n, dtype=ld)
    w = [R @ cheb_second_derivative(np.asarray(g, dtype=ld)) for g in bc]
    lin = cheb_to_ct_closed(n, 2, dtype=ld)  # C~ coefficients of T_0, T_1
    am = lin @ np.array([0.5, -0.5], dtype=ld)  # (1 - t)/2
    ap = lin @ np.array([0.5, 0.5], dtype=ld)   # (1 + t)/2
    L, Rt, B, T = w
    C = (ld(sx2) * (np.outer(am, B) + np.outer(ap, T))
         + ld(sy2) * (np.outer(L, am) + np.outer(Rt, ap)))
    return C.astype(np.float64)


def lift_correction_2d(bc, box, n: int) -> np.ndarray:
    """The same correction from its definition in two dimensions, in float64:
    the C~ projection of the Chebyshev coefficients of Lap u_bc (accurate for
    smooth traces and small n; the cross-check of lift_correction)."""
    return ct_projection(laplacian_coeffs(coons_coeffs(bc), box), n)


def poisson_rect_dirichlet(F_T: np.ndarray, bc, box) -> np.ndarray:
    """U ((n+2) x (n+2) Chebyshev coefficients) of Lap u = f on the box with
    u = the given traces on the boundary (Sec. 6.1): u = u0 + u_bc with
    u_bc the transfinite interpolant of the traces and u0 the zero-data
    discrete solution for the right-hand side f - Lap u_bc."""
    n = F_T.shape[0]
    Ubc = coons_coeffs(bc)
    assert Ubc.shape == (n + 2, n + 2)
    F_C = rhs_ct(F_T) - lift_correction(bc, box, n)
    U0 = to_chebyshev(solve_native_rect(F_C, box))
    return U0 + Ubc


def boundary_traces(U: np.ndarray):
    """(L, R, B, T) coefficient vectors of u(-1, t), u(1, t), u(s, -1), u(s, 1)."""
    k = np.arange(U.shape[1])
    j = np.arange(U.shape[0])
    L = U @ ((-1.0) ** k)
    R = U @ np.ones(U.shape[1])
    B = ((-1.0) ** j) @ U
    T = np.ones(U.shape[0]) @ U
    return L, R, B, T
