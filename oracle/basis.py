"""Ultraspherical basis, discretization matrices and coefficient maps.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper passages:
* Sec. 3.1, footnote: C~_j = sqrt((j+3/2)/((j+1)(j+2))) C_j^(3/2), so that
  int_{-1}^{1} C~_j(x)^2 (1-x^2) dx = 1.
* (3.4) and the display after it: ((1-x^2) C~_j)'' = -(j(j+3)+2) C~_j.
* (3.6): M X D^T + D X M^T = F with D_jj = -(j(j+3)+2) and M the matrix of
  multiplication by (1-x^2) in the C~ basis, entries (3.7).
* Sec. 3.4: the right-hand side must be given in C~ coefficients; the solution
  u = sum X_ij (1-y^2)(1-x^2) C~_i(y) C~_j(x) is a polynomial of degree n+1 in
  each variable, so its Chebyshev coefficients form an (n+2) x (n+2) array.
"""
from __future__ import annotations

import numpy as np
import scipy.special as sps


def ct_values(n: int, x: np.ndarray) -> np.ndarray:
    """C~_j(x) for j = 0..n-1, shape (n, len(x)).

    Unnormalized C_j^(3/2) from the three-term recurrence of the Gegenbauer
    polynomials (NIST 18.9.1 with lambda = 3/2):
        (k+1) C_{k+1} = (2k+3) x C_k - (k+2) C_{k-1},  C_0 = 1, C_1 = 3x,
    then the normalization of the Sec. 3.1 footnote."""
    x = np.asarray(x, dtype=np.float64)
    C = np.zeros((n, x.size))
    if n == 0:
        return C
    C[0] = 1.0
    if n > 1:
        C[1] = 3.0 * x
    for k in range(1, n - 1):
        C[k + 1] = ((2 * k + 3) * x * C[k] - (k + 2) * C[k - 1]) / (k + 1)
    j = np.arange(n, dtype=np.float64)
    return C * np.sqrt((j + 1.5) / ((j + 1) * (j + 2)))[:, None]


def gauss_jacobi11(N: int):
    """N-point Gauss quadrature for the weight (1-x^2) on [-1, 1]."""
    x, w = sps.roots_jacobi(N, 1.0, 1.0)
    return x, w


def D_diag(n: int) -> np.ndarray:
    """Diagonal of D in (3.6): D_jj = -(j(j+3)+2)."""
    j = np.arange(n, dtype=np.float64)
    return -(j * (j + 3) + 2)


def mult_M(n: int, rows: int | None = None) -> np.ndarray:
    """Multiplication by (1-x^2) in the C~ basis, entries (3.7).

    Column j holds the C~ coefficients of (1-x^2) C~_j, which are nonzero at
    rows j-2, j, j+2.  ``rows`` = n gives the square n x n matrix of (3.6);
    rows = n + 2 keeps the two extra degrees (used for the solution's
    coefficients, which reach degree n+1)."""
    rows = n if rows is None else rows
    M = np.zeros((rows, n))
    for j in range(max(rows, n)):
        jj = float(j)
        diag = 2 * (jj + 1) * (jj + 2) / ((2 * jj + 1) * (2 * jj + 5))
        fact = 1.0
        for t in range(1, 5):
            fact *= jj + t  # (j+4)!/j!
        off = -1.0 / ((2 * jj + 3) * (2 * jj + 5)) * np.sqrt(fact * (2 * jj + 3) / (2 * jj + 7))
        if j < rows and j < n:
            M[j, j] = diag
        # M_{j,j+2} = M_{j+2,j}: (1-x^2) C~_j has C~_{j+2} component, and
        # (1-x^2) C~_{j+2} has a C~_j component, both equal by symmetry.
        if j < rows and j + 2 < n:
            M[j, j + 2] = off
        if j + 2 < rows and j < n:
            M[j + 2, j] = off
    return M


def cheb_T(n: int, x: np.ndarray) -> np.ndarray:
    """T_k(x) for k = 0..n-1, shape (n, len(x)), as cos(k arccos x)."""
    x = np.clip(np.asarray(x, dtype=np.float64), -1.0, 1.0)
    return np.cos(np.outer(np.arange(n), np.arccos(x)))


def cheb_to_ct(n: int) -> np.ndarray:
    """R with R[i, k] = int T_k(x) C~_i(x) (1-x^2) dx, i.e. column k holds the
    C~ coefficients of T_k (orthonormality of C~ under (1-x^2), footnote of
    Sec. 3.1), for i, k < n, entrywise from the Gegenbauer connection formula
    (DLMF 18.18.16) in the limit that gives T_k (DLMF 18.7.25), mu = 3/2:
      T_k = (k/2) sum_l A(k-l) B(l) (k - 2l + mu) C^(mu)_{k-2l},
      A(j) = (j-1)! / (mu)_{j+1},  B(l) = (-mu)_l / l!,
    with C^(mu)_i = C~_i / nu_i.  A and B are tabulated once in extended
    precision by their ratio recurrences, so every entry is a product of a
    few accurately known factors (relative accuracy of a few eps; Gauss-Jacobi
    quadrature of the integrals in float64 leaves absolute errors ~ eps that
    grow relative to the small entries with n: 9e-14 relative at n = 512)."""
    R = np.zeros((n, n))
    if n == 0:
        return R
    ld = np.longdouble
    mu = ld(1.5)
    j = np.arange(1, n + 1).astype(ld)
    # A(1) = 1/(mu (mu+1)), A(j+1)/A(j) = j/(mu + j + 1); index j - 1
    A = np.cumprod(np.concatenate([[1 / (mu * (mu + 1))], j[:-1] / (mu + j[:-1] + 1)])).astype(np.float64)
    l_ = np.arange(n).astype(ld)
    # B(0) = 1, B(l+1)/B(l) = (l - mu)/(l + 1)
    B = np.cumprod(np.concatenate([[ld(1)], (l_[:-1] - mu) / (l_[:-1] + 1)])).astype(np.float64)
    i_all = np.arange(n, dtype=np.float64)
    nu = np.sqrt((i_all + 1.5) / ((i_all + 1) * (i_all + 2)))
    RT = np.zeros((n, n))  # row k holds column k (returned transposed, no copy)
    RT[0, 0] = 1 / nu[0]   # T_0 = C^(mu)_0
    for k in range(1, n):
        l = np.arange(k // 2 + 1)
        i = k - 2 * l
        RT[k, i] = (k / 2) * A[k - l - 1] * B[l] * (i + 1.5) / nu[i]
    return RT.T


def cheb_points(N: int) -> np.ndarray:
    """First-kind Chebyshev points cos((m+1/2) pi / N), m = 0..N-1."""
    return np.cos((np.arange(N) + 0.5) * np.pi / N)


def dct_matrix(N: int) -> np.ndarray:
    """Matrix taking values at the N first-kind points to the Chebyshev
    coefficients of the degree-(N-1) interpolant (discrete orthogonality of
    cos(k theta) on the points)."""
    m = np.arange(N)
    C = np.cos(np.outer(np.arange(N), (m + 0.5) * np.pi / N)) * (2.0 / N)
    C[0] *= 0.5
    return C


def recombined_to_cheb(n: int) -> np.ndarray:
    """P (n+2) x n with column i = Chebyshev coefficients of (1-x^2) C~_i(x)
    (the expansion (3.2)), entrywise from a closed form:
      * C^(3/2)_i = P'_{i+1} (NIST 18.9.19 with lambda = 1/2) and
        (1-x^2) P'_{i+1} = (i+1)(i+2)/(2i+3) (P_i - P_{i+2}) (Legendre P),
      * P_m = sum_{k <= m, k = m mod 2} (2 - [k = 0])/pi L((m-k)/2) L((m+k)/2) T_k
        with L(z) = Gamma(z + 1/2)/Gamma(z + 1) (the Legendre-to-Chebyshev
        connection, DLMF 18.18.16 at lambda = 1/2 in the limit mu -> 0),
      * L(z + 1) = L(z) (z + 1/2)/(z + 1), so for k <= i, a = (i-k)/2,
        b = (i+k)/2 the two terms combine without cancellation:
          coefficient = nu_i (i+1)(i+2)/4 (2 - [k = 0])/pi L(a) L(b) / ((a+1)(b+1)),
        and T_{i+2} takes -nu_i (i+1)(i+2)/(2i+3) (2/pi) L(0) L(i+2),
    with C~_i = nu_i C^(3/2)_i (footnote of Sec. 3.1).  Every factor is
    positive, so each entry has relative accuracy of a few eps (sampling at
    n+2 points and a float64 DCT gives the same matrix with rounding that
    grows with n: 3.4e-14 relative at n = 512)."""
    N = n + 2
    if n == 0:
        return np.zeros((N, n))
    # L(m) for integer m = 0 .. n+1 by the ratio recurrence, in extended precision
    ld = np.longdouble
    m = np.arange(n + 2)
    ratios = (m[:-1].astype(ld) + ld(0.5)) / (m[:-1].astype(ld) + 1)
    L = np.concatenate([[np.sqrt(ld(np.pi))], np.sqrt(ld(np.pi)) * np.cumprod(ratios)]).astype(np.float64)
    PT = np.zeros((n, N))  # row i holds column i (returned transposed, no copy)
    for i in range(n):
        nu = np.sqrt((i + 1.5) / ((i + 1) * (i + 2)))
        k = np.arange(i % 2, i + 1, 2)
        a, b = (i - k) // 2, (i + k) // 2
        w = np.where(k == 0, 1.0, 2.0) / np.pi
        PT[i, k] = nu * (i + 1) * (i + 2) / 4 * w * L[a] * L[b] / ((a + 1.0) * (b + 1.0))
        PT[i, i + 2] = -nu * (i + 1) * (i + 2) / (2 * i + 3) * (2 / np.pi) * L[0] * L[i + 2]
    return PT.T


def cheb_eval_2d(U: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """u(x_m, y_m) = sum_{j,k} U[j, k] T_j(y_m) T_k(x_m) at matching points."""
    Ty = cheb_T(U.shape[0], y)
    Tx = cheb_T(U.shape[1], x)
    return np.einsum("jm,jk,km->m", Ty, U, Tx)
