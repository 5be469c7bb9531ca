"""Pins for oracle.cylinder: spectral convergence to a manufactured solution on
the cylinder (through the DFS doubling, the three mode cases and the output
maps), brute-force Kronecker solves against Bartels-Stewart, the derivative
identities of the basis, and the failure of the printed L1 / A formulas
(which is why the oracle follows (4.8) instead)."""
import numpy as np
import pytest

import workloads
from oracle import basis, cylinder


def _max_err(n, N=96, seed=0):
    F, ufun, _ = workloads.manufactured_cylinder(n, n, N)
    U = cylinder.poisson_cylinder(F)
    rng = np.random.default_rng(seed)
    r, th, z = rng.uniform(0, 1, 40), rng.uniform(-np.pi, np.pi, 40), rng.uniform(-1, 1, 40)
    ue = cylinder.evaluate(U, r, th, z)
    return np.abs(ue - ufun(r * np.cos(th), r * np.sin(th), z)).max()


def test_manufactured_solution_spectral_convergence():
    errs = [_max_err(n) for n in (8, 16, 28, 40)]
    assert errs[-1] < 1e-12
    assert errs[0] > 100 * errs[1] > 1e4 * errs[2]


def test_manufactured_rhs_is_the_laplacian():
    # central differences of u against the written-out f
    _, u, f = workloads.manufactured_cylinder(4, 4, 8)
    rng = np.random.default_rng(1)
    h = 1e-3
    for x, y, z in rng.uniform(-0.6, 0.6, (6, 3)):
        p = np.array([x, y, z])
        lap = sum((u(*(p + h * e)) - 2 * u(*p) + u(*(p - h * e))) / h ** 2 for e in np.eye(3))
        assert abs(lap - f(x, y, z)) < 1e-5 * max(1.0, abs(f(x, y, z)))


@pytest.mark.parametrize("n", [4, 8, 10])
def test_bartels_stewart_matches_kronecker(n):
    F = workloads.cylinder_rhs(n, 8, seed=n)
    U1 = cylinder.poisson_cylinder(F, method="kron")
    U2 = cylinder.poisson_cylinder(F, method="bs")
    assert np.abs(U1 - U2).max() <= 1e-13 * np.abs(U1).max()


def test_basis_derivatives_satisfy_3_4():
    # ((1 - x^2) C~_j)'' = -(j(j+3)+2) C~_j  ((3.4)) from the derivative values
    n = 30
    x = np.linspace(-0.99, 0.99, 41)
    c0, c1, c2 = cylinder.ct_and_derivatives(n, x)
    lhs = (1 - x * x)[None, :] * c2 - 4 * x[None, :] * c1 - 2 * c0
    rhs = basis.D_diag(n)[:, None] * c0
    assert np.abs(lhs - rhs).max() < 1e-9 * np.abs(rhs).max()
    # C~ itself against the square's basis routine
    assert np.abs(c0 - basis.ct_values(n, x)).max() < 1e-12


def test_galerkin_multiplication_matrices():
    n = 20
    M = cylinder.galerkin(n, lambda c0, c1, c2, r: (1 - r * r) * c0)
    assert np.abs(M - basis.mult_M(n)).max() < 1e-14
    Mr2 = cylinder.galerkin(n, lambda c0, c1, c2, r: r * r * c0)
    assert np.abs(M + Mr2 - np.eye(n)).max() < 1e-13


def test_solution_parity_and_real_data():
    n, nt = 12, 10
    F, _, _ = workloads.manufactured_cylinder(n, nt, 48)
    U = cylinder.poisson_cylinder(F)
    ks = np.arange(nt) - nt // 2
    for idx, k in enumerate(ks):
        wrong = np.arange((abs(k) + 1) % 2, n + 4, 2)
        assert np.abs(U[idx][wrong, :]).max() < 1e-14 * max(1.0, np.abs(U[idx]).max())
    # a real f gives U_{-k} = conj(U_k)
    for idx, k in enumerate(ks):
        if k != -nt // 2:
            j = nt // 2 - k
            assert np.abs(U[idx] - np.conj(U[j])).max() < 1e-12


def test_printed_l1_formula_does_not_converge():
    # replacing the zeroth-order term 4(1 - 4 r^2) of (4.8) by the 8 - 16 r^2
    # that the printed matrix formula gives destroys convergence
    n = 28
    F, ufun, _ = workloads.manufactured_cylinder(n, n, 96)
    orig = cylinder.mode_operators

    def printed(nn, k):
        P, Q, Mr2, m, wp, rp = orig(nn, k)
        if cylinder.mode_case(k) == 1:
            P = P + cylinder.galerkin(nn, lambda c0, c1, c2, r: 4 * c0)
        return P, Q, Mr2, m, wp, rp

    cylinder.mode_operators = printed
    try:
        U = cylinder.poisson_cylinder(F)
    finally:
        cylinder.mode_operators = orig
    rng = np.random.default_rng(0)
    r, th, z = rng.uniform(0, 1, 40), rng.uniform(-np.pi, np.pi, 40), rng.uniform(-1, 1, 40)
    err = np.abs(cylinder.evaluate(U, r, th, z) - ufun(r * np.cos(th), r * np.sin(th), z)).max()
    assert err > 1e-4
