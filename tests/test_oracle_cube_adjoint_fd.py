"""Pins for oracle.cube, oracle.adjoint and the shift machinery on the
finite-difference problem (1.2)-(1.3)."""
import numpy as np
import pytest
import sympy as sy

import workloads
from oracle import adjoint, basis, cube, fd, shifts, square


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n", [1, 3, 6])
def test_cube_eigen_matches_kronecker(n):
    rng = np.random.default_rng(10 + n)
    F_C = rng.standard_normal((n, n, n))
    assert _rel(cube.solve_native(F_C), cube.kron_solve(F_C)) < 1e-12


def test_cube_sign_and_scaling_from_laplacian_identity():
    # build f = Lap u symbolically for u = (1-x^2)(1-y^2)(1-z^2) C~_1(z) C~_0(y) C~_2(x)
    # and check the cube solve returns exactly that single coefficient.
    x, y, z = sy.symbols("x y z")
    def ct(j, t):
        return sy.sqrt(sy.Rational(2 * j + 3, 2) / ((j + 1) * (j + 2))) * sy.gegenbauer(j, sy.Rational(3, 2), t)
    u = (1 - x ** 2) * (1 - y ** 2) * (1 - z ** 2) * ct(1, z) * ct(0, y) * ct(2, x)
    f = sy.diff(u, x, 2) + sy.diff(u, y, 2) + sy.diff(u, z, 2)
    n = 5
    F = workloads.cheb_coeffs_3d(sy.lambdify((x, y, z), f, "numpy"), n)
    X = cube.solve_native(cube.rhs_ct(F))
    ref = np.zeros((n, n, n))
    ref[1, 0, 2] = 1.0
    assert np.abs(X - ref).max() < 1e-13


def test_cube_manufactured_convergence():
    errs = []
    for n in (8, 14, 20):
        F, u_fun = workloads.manufactured_cube(n, N=40)
        U = cube.poisson_cube(F)
        Uex = workloads.cheb_coeffs_3d(u_fun, n + 2)
        errs.append(np.abs(U - Uex).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[-1] < 1e-12


def test_adjoint_dot_product_exact_and_adi():
    n = 18
    rng = np.random.default_rng(0)
    F = rng.standard_normal((n, n))
    Ub = rng.standard_normal((n + 2, n + 2))
    lhs = np.sum(square.poisson_square(F) * Ub)
    rhs = np.sum(F * adjoint.vjp_square(Ub))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    _, p, _ = shifts.square_shifts(n, 1e-6)
    lhs = np.sum(square.poisson_square_adi(F, p) * Ub)
    rhs = np.sum(F * adjoint.vjp_square(Ub, p))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_adjoint_central_difference_of_quadratic_loss():
    n = 12
    rng = np.random.default_rng(1)
    F = rng.standard_normal((n, n))
    target = rng.standard_normal((n + 2, n + 2))
    loss = lambda FF: np.sum((square.poisson_square(FF) - target) ** 2)  # noqa: E731
    grad = adjoint.vjp_square(2 * (square.poisson_square(F) - target))
    h = 1e-6
    for _ in range(4):
        dirn = rng.standard_normal((n, n))
        dirn /= np.linalg.norm(dirn)
        fdv = (loss(F + h * dirn) - loss(F - h * dirn)) / (2 * h)
        assert abs(fdv - np.sum(grad * dirn)) < 1e-7 * max(1.0, abs(fdv))


@pytest.mark.parametrize("n", [16, 64])
def test_adi_on_fd_problem_matches_sine_transform(n):
    # Sec. 2.1: ADI with the Theorem 2.1 shifts on K X + X K^T = F over the
    # intervals [-n^2, -1], [1, n^2] reproduces the DST-I solution (1.3).
    rng = np.random.default_rng(n)
    F = rng.standard_normal((n - 1, n - 1))
    K = fd.K_matrix(n)
    tol = 1e-10
    J, p, q = shifts.zolotarev_shifts(*fd.enclosure(n), tol=tol)
    X = square.adi_dense(K, -K.T, F, p, q)
    Xd = fd.dst_solve(F)
    assert np.linalg.norm(X - Xd, 2) <= 10 * tol * np.linalg.norm(Xd, 2)
    ev = np.linalg.eigvalsh(K)
    assert ev.min() >= -n ** 2 and ev.max() <= -1
