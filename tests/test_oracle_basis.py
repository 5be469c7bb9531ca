"""Pins for oracle.basis against symbolic integration, library routines and
function-value identities (CPU only)."""
import numpy as np
import pytest
import scipy.special as sps
import sympy as sy

from oracle import basis

x_ = sy.Symbol("x")


def _ct_sym(j):
    # normalized C~_j^(3/2) from sympy's Gegenbauer polynomial (footnote, Sec. 3.1)
    return sy.sqrt(sy.Rational(2 * j + 3, 2) / ((j + 1) * (j + 2))) * sy.gegenbauer(j, sy.Rational(3, 2), x_)


def test_ct_values_match_scipy_gegenbauer():
    x = np.linspace(-1, 1, 37)
    V = basis.ct_values(30, x)
    for j in range(30):
        ref = sps.eval_gegenbauer(j, 1.5, x) * np.sqrt((j + 1.5) / ((j + 1) * (j + 2)))
        assert np.allclose(V[j], ref, rtol=1e-13, atol=1e-13)


def test_ct_orthonormal_under_weight():
    n = 48
    xq, wq = basis.gauss_jacobi11(n + 2)
    V = basis.ct_values(n, xq)
    Gram = (V * wq) @ V.T
    assert np.abs(Gram - np.eye(n)).max() < 1e-13


@pytest.mark.parametrize("j", range(7))
def test_eigen_relation_3_4_symbolic(j):
    # ((1-x^2) C~_j)'' = -(j(j+3)+2) C~_j  (display after (3.4))
    c = _ct_sym(j)
    lhs = sy.diff((1 - x_ ** 2) * c, x_, 2)
    assert sy.simplify(lhs + (j * (j + 3) + 2) * c) == 0


def test_mult_matrix_3_7_against_exact_gram():
    # M_lj = int (1-x^2) C~_j C~_l (1-x^2) dx, exact rational/surd arithmetic
    n = 8
    M = basis.mult_M(n)
    for l in range(n):
        for j in range(n):
            val = sy.integrate((1 - x_ ** 2) ** 2 * _ct_sym(j) * _ct_sym(l), (x_, -1, 1))
            assert abs(float(val) - M[l, j]) < 1e-15, (l, j)


def test_rectangular_M_columns_expand_product():
    # (1-x^2) C~_j(x) = sum_l M[l, j] C~_l(x) with l up to n+1 (rows n+2)
    n = 20
    M = basis.mult_M(n, rows=n + 2)
    x = np.linspace(-0.99, 0.99, 41)
    lhs = (1 - x ** 2)[None, :] * basis.ct_values(n, x)
    rhs = M.T @ basis.ct_values(n + 2, x)
    assert np.abs(lhs - rhs).max() < 1e-12


def test_D_diag():
    assert list(basis.D_diag(4)) == [-2.0, -6.0, -12.0, -20.0]


def test_cheb_to_ct_reproduces_function_values():
    rng = np.random.default_rng(5)
    n = 60
    c = rng.standard_normal(n)
    R = basis.cheb_to_ct(n)
    x = rng.uniform(-1, 1, 50)
    f_T = c @ basis.cheb_T(n, x)
    f_C = (R @ c) @ basis.ct_values(n, x)
    assert np.abs(f_T - f_C).max() < 1e-12 * np.abs(c).sum()
    # upper triangular with parity structure
    i, k = np.indices(R.shape)
    assert np.all(R[(i > k) | ((k - i) % 2 == 1)] == 0) or \
        np.abs(R[(i > k) | ((k - i) % 2 == 1)]).max() < 1e-14


def test_recombined_to_cheb_matches_direct_expansion():
    n = 30
    P = basis.recombined_to_cheb(n)
    x = np.linspace(-1, 1, 53)
    lhs = (1 - x ** 2)[None, :] * basis.ct_values(n, x)
    rhs = P.T @ basis.cheb_T(n + 2, x)
    assert np.abs(lhs - rhs).max() < 1e-12


@pytest.mark.parametrize("n", [1, 2, 7, 64])
def test_cheb_to_ct_equals_its_integral_definition(n):
    # R[i, k] = int T_k C~_i (1 - x^2) dx by Gauss-Jacobi quadrature (exact for
    # the degree 2n - 2 integrand at these n): the closed form must agree
    x, w = basis.gauss_jacobi11(n + 1)
    Rq = (basis.ct_values(n, x) * w[None, :]) @ basis.cheb_T(n, x).T
    R = basis.cheb_to_ct(n)
    assert np.abs(R - Rq).max() < 1e-14 * max(1.0, np.abs(Rq).max())


@pytest.mark.parametrize("n", [1, 2, 7, 64])
def test_recombined_to_cheb_equals_interpolation(n):
    # the degree-(n+1) functions (1 - x^2) C~_i are interpolated exactly on
    # n + 2 first-kind points: sampling + discrete cosine map gives P too
    N = n + 2
    x = basis.cheb_points(N)
    Ps = basis.dct_matrix(N) @ ((1 - x * x)[None, :] * basis.ct_values(n, x)).T
    P = basis.recombined_to_cheb(n)
    assert np.abs(P - Ps).max() < 1e-14 * max(1.0, np.abs(Ps).max())
