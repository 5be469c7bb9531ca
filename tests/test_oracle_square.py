"""Pins for oracle.square: brute-force Kronecker solves, the spectrum of A~
(Lemma B.1 and the continuum limit), Algorithm 2 against its closed form,
the P1 error bound, manufactured solutions and the (3.9) reading."""
import json
import os

import numpy as np
import pytest

import workloads
from oracle import basis, shifts, square

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_paper_n1_value():
    with open(os.path.join(GOLD, "paper_values.json")) as f:
        gold = json.load(f)
    A = square.atilde_dense(1)
    assert abs(A[0, 0] - gold["atilde_n1"]["value"]) < 1e-15


@pytest.mark.parametrize("n", [1, 2, 5, 12, 30])
def test_eigen_solve_matches_kronecker(n):
    rng = np.random.default_rng(n)
    F_C = rng.standard_normal((n, n))
    X = square.solve_native(F_C)
    Xk = square.kron_solve_generalized(F_C)
    assert _rel(X, Xk) < 1e-13


def test_residual_of_generalized_sylvester():
    n = 64
    F_C = square.rhs_ct(workloads.square_rhs(n))
    X = square.solve_native(F_C)
    M = basis.mult_M(n)
    D = np.diag(basis.D_diag(n))
    assert _rel(M @ X @ D + D @ X @ M, F_C) < 1e-13


def test_literal_3_9_transform_is_wrong_and_congruence_is_right():
    # Y = D_s^-1 X D_s (as printed) does not solve A~ Y - Y B~ = G; the
    # congruence Y = D_s^-1 X D_s^-1 with D_s = S^-1 does.
    n = 12
    rng = np.random.default_rng(3)
    F_C = rng.standard_normal((n, n))
    X = square.solve_native(F_C)
    s = square.s_diag(n)
    A = square.atilde_dense(n)
    G = F_C / np.outer(s, s)
    Y_cong = X * np.outer(s, s)
    Y_lit = X * np.outer(s, 1.0 / s)
    assert _rel(A @ Y_cong + Y_cong @ A, G) < 1e-13
    assert _rel(A @ Y_lit + Y_lit @ A, G) > 1e-2


@pytest.mark.parametrize("n", [1, 2, 5, 16, 64, 200])
def test_lemma_b1_spectrum(n):
    lam, _ = square.atilde_eig(n)
    assert lam.min() > -1.0
    assert lam.max() < -1.0 / (30.0 * n ** 4)
    if n > 1:
        assert lam.max() < -3.0 / (64 * n ** 4) + 1.0 / (64 * n ** 5)


def test_spectrum_continuum_limit():
    # M v = lam D v is the discretization of w = lam w'', w(+-1) = 0, whose
    # eigenvalues are -4/(k pi)^2 (textbook Dirichlet problem on [-1, 1]).
    lam, _ = square.atilde_eig(200)
    top = np.sort(lam)[:4]
    ref = -4.0 / (np.pi * np.arange(1, 5)) ** 2
    assert np.allclose(top, ref, rtol=1e-8)


def test_atilde_entries_against_closed_form():
    n = 40
    A = square.atilde_dense(n)
    j = np.arange(n)
    assert np.allclose(np.diag(A), -2.0 / ((2 * j + 1) * (2 * j + 5)), rtol=1e-15)
    jj = j[: n - 2]
    assert np.allclose(np.diag(A, 2), 1.0 / ((2 * jj + 5) * np.sqrt((2 * jj + 3) * (2 * jj + 7))), rtol=1e-14)
    assert np.all(np.diag(A, 1) == 0)


def test_algorithm2_dense_equals_closed_form():
    n = 20
    G = workloads.square_rhs(n, seed=7)
    J, p, q = shifts.square_shifts(n, 1e-8)
    A = square.atilde_dense(n)
    Yd = square.adi_dense(A, -A, G, p, q)
    Yc = square.adi_exact_iterate(G, p)
    assert _rel(Yd, Yc) < 1e-11
    # and the J-step error obeys the P1 bound of Theorem 2.1
    Y = square.solve_symmetric_sylvester(G)
    err = np.linalg.norm(Y - Yc, 2) / np.linalg.norm(Y, 2)
    g = shifts.cross_ratio(*shifts.square_enclosure(n))
    assert err <= shifts.zolotarev_bound(g, J) <= 1e-8


def test_closed_form_with_few_shifts_is_not_converged():
    n = 30
    G = workloads.square_rhs(n, seed=1)
    _, p, _ = shifts.square_shifts(n, 1e-1)
    Y = square.solve_symmetric_sylvester(G)
    assert _rel(square.adi_exact_iterate(G, p), Y) > 1e-6


def test_manufactured_solution_spectral_convergence():
    # u = (1-x^2)(1-y^2) exp(sin 3x cos 2y): the discrete solution converges
    # spectrally to the exact Chebyshev coefficients of u.
    errs = []
    for n in (16, 24, 32, 48):
        F, u_fun = workloads.manufactured_square(n, N=96)
        U = square.poisson_square(F)
        Uex = workloads.cheb_coeffs_2d(u_fun, n + 2)
        errs.append(np.abs(U - Uex).max())
    assert errs[-1] < 1e-13
    assert errs[0] > errs[1] > errs[2]


def test_orientation_rows_are_y():
    # rows <-> y: swapping x and y in f transposes F and must transpose U;
    # a y-only right-hand side gives an x-y asymmetric solution.  (Absolute
    # orientation is pinned by the x-y asymmetric manufactured solution.)
    n = 10
    F = np.zeros((n, n))
    F[2, 0] = 1.0
    U = square.poisson_square(F)
    assert np.abs(U - U.T).max() > 1e-3
    assert np.abs(square.poisson_square(F.T) - U.T).max() < 1e-15


def test_dirichlet_boundary_zero():
    n = 24
    U = square.poisson_square(workloads.square_rhs(n, seed=2))
    t = np.linspace(-1, 1, 17)
    one = np.ones_like(t)
    for xx, yy in ((one, t), (-one, t), (t, one), (t, -one)):
        assert np.abs(basis.cheb_eval_2d(U, xx, yy)).max() < 1e-14
