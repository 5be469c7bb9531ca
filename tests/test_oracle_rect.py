"""Pins for oracle.rect: the rectangle system against a brute-force Kronecker
solve, the Galerkin conditions checked by quadrature of point values, a
manufactured solution with nonzero boundary values on a non-square box, the
boundary-trace identity of the Dirichlet lift, reductions to the square, and
Algorithm 2 with the rectangle's general-interval shifts against its closed
form and the bound of Theorem 2.1."""
import numpy as np
import pytest

import workloads
from oracle import basis, rect, shifts, square

BOX = (0.0, 2.5, -1.0, 0.25)  # sx^2 = 0.64, sy^2 = 2.56


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n", [1, 2, 5, 12, 25])
def test_eigen_solve_matches_kronecker(n):
    rng = np.random.default_rng(n + 100)
    F_C = rng.standard_normal((n, n))
    assert _rel(rect.solve_native_rect(F_C, BOX), rect.kron_solve_rect(F_C, BOX)) < 1e-13


def test_unit_box_reduces_to_square():
    n = 33
    F = workloads.square_rhs(n, seed=3)
    U = rect.poisson_rect(F, (-1.0, 1.0, -1.0, 1.0))
    assert _rel(U, square.poisson_square(F)) < 1e-14


def test_scaling_of_a_square_box():
    # on [-L, L]^2, u(x, y) = L^2 u1(x/L, y/L) where Lap u1 = f(L s, L t):
    # in mapped coefficients U = L^2 U1 for the same F.
    n, Lh = 21, 3.0
    F = workloads.square_rhs(n, seed=4)
    U = rect.poisson_rect(F, (-Lh, Lh, -Lh, Lh))
    assert _rel(U, Lh ** 2 * square.poisson_square(F)) < 1e-14


def _galerkin_residual(U, F, n):
    """max |int int (Lap u - f) C~_k(t) C~_l(s) (1-s^2)(1-t^2)| over k, l < n,
    by tensor Gauss-Jacobi quadrature of point values (exact: degree <= 2n)."""
    x, w = basis.gauss_jacobi11(2 * n + 4)
    P = basis.ct_values(n, x) * w[None, :]
    LU = rect.laplacian_coeffs(U, BOX)

    def vals(C):
        return basis.cheb_T(C.shape[0], x).T @ C @ basis.cheb_T(C.shape[1], x)

    Rg = P @ (vals(LU) - vals(F)) @ P.T
    return np.abs(Rg).max() / np.abs(P @ vals(F) @ P.T).max()


def test_galerkin_conditions_by_quadrature():
    # Lap u has degree n+1 in each variable; the discretization asks that
    # Lap u - f be orthogonal to C~_k C~_l (k, l < n) under the weight.
    n = 40
    F = workloads.square_rhs(n, seed=8)
    U = rect.poisson_rect(F, BOX)
    assert _galerkin_residual(U, F, n) < 1e-10
    # and the conditions are not empty: Lap u != f as polynomials
    assert _rel(rect.laplacian_coeffs(U, BOX)[:n, :n], F) > 1e-6


def test_galerkin_equations_against_transposed_box():
    # swapping x and y swaps the box sides and transposes F and U
    n = 17
    F = workloads.square_rhs(n, seed=9)
    a, b, c, d = BOX
    U = rect.poisson_rect(F, BOX)
    Ut = rect.poisson_rect(F.T, (c, d, a, b))
    assert _rel(Ut, U.T) < 1e-14


def test_dirichlet_traces_are_reproduced():
    n = 30
    F, bc = workloads.rect_dirichlet_case(n, seed=5)
    U = rect.poisson_rect_dirichlet(F, bc, BOX)
    assert U.shape == (n + 2, n + 2)
    for got, want in zip(rect.boundary_traces(U), bc):
        assert np.abs(got - want).max() < 1e-13 * np.abs(bc).max()
    assert _galerkin_residual(U, F, n) < 1e-10


def test_coons_lift_pointwise():
    # the transfinite interpolant agrees with each trace on its edge and is
    # bilinear-corrected: check by evaluation at points along all four edges
    n = 12
    _, bc = workloads.rect_dirichlet_case(n, seed=11)
    Ubc = rect.coons_coeffs(bc)
    t = np.linspace(-1, 1, 23)
    one = np.ones_like(t)
    L, R, B, T = bc
    from numpy.polynomial import chebyshev as npc
    assert np.abs(basis.cheb_eval_2d(Ubc, -one, t) - npc.chebval(t, L)).max() < 1e-13
    assert np.abs(basis.cheb_eval_2d(Ubc, one, t) - npc.chebval(t, R)).max() < 1e-13
    assert np.abs(basis.cheb_eval_2d(Ubc, t, -one) - npc.chebval(t, B)).max() < 1e-13
    assert np.abs(basis.cheb_eval_2d(Ubc, t, one) - npc.chebval(t, T)).max() < 1e-13


def test_zero_data_reduces_to_homogeneous_solve():
    n = 19
    F = workloads.square_rhs(n, seed=12)
    U = rect.poisson_rect_dirichlet(F, np.zeros((4, n + 2)), BOX)
    assert _rel(U, rect.poisson_rect(F, BOX)) < 1e-15


def test_harmonic_polynomial_is_recovered():
    # u = x^2 - y^2 + 3xy in physical coordinates is harmonic: with f = 0 and
    # its traces, the solution is u itself (degree 2 fits any n >= 1).
    a, b, c, d = BOX
    n = 6

    def u(s, t):
        x = (a + b) / 2 + (b - a) / 2 * s
        y = (c + d) / 2 + (d - c) / 2 * t
        return x * x - y * y + 3 * x * y

    N = n + 2
    p = basis.cheb_points(N)
    one = np.ones(N)
    Dm = basis.dct_matrix(N)
    bc = np.stack([Dm @ u(-one, p), Dm @ u(one, p), Dm @ u(p, -one), Dm @ u(p, one)])
    U = rect.poisson_rect_dirichlet(np.zeros((n, n)), bc, BOX)
    Uex = workloads.cheb_coeffs_2d(u, N)
    assert np.abs(U - Uex).max() < 1e-13


def test_manufactured_nonzero_boundary_spectral_convergence():
    errs = []
    for n in (4, 6, 8, 10, 12, 24):
        F, bc, u_fun = workloads.manufactured_rect(n, BOX)
        U = rect.poisson_rect_dirichlet(F, bc, BOX)
        Uex = workloads.cheb_coeffs_2d(u_fun, n + 2)
        errs.append(np.abs(U - Uex).max())
    assert errs[-1] < 1e-13
    assert all(e1 > 50 * e2 for e1, e2 in zip(errs[:5], errs[1:5]))
    # pointwise at random points
    rng = np.random.default_rng(0)
    s, t = rng.uniform(-1, 1, 50), rng.uniform(-1, 1, 50)
    assert np.abs(basis.cheb_eval_2d(U, s, t) - u_fun(s, t)).max() < 1e-12


def test_rect_enclosure_contains_spectra():
    n = 40
    lam, _ = square.atilde_eig(n)
    a, b, c, d = rect.rect_enclosure(n, BOX)
    sx2, sy2 = rect.scalings(BOX)
    assert a <= (sx2 * lam).min() and (sx2 * lam).max() <= b
    assert c <= (-sy2 * lam).min() and (-sy2 * lam).max() <= d
    assert b < 0 < c


def test_algorithm2_dense_equals_closed_form_on_rectangle():
    n = 18
    G = workloads.square_rhs(n, seed=13)
    J, p, q = rect.rect_shifts(n, BOX, 1e-9)
    A, B = rect.rect_operators(n, BOX)
    Yd = square.adi_dense(A, B, G, p, q)
    Yc = rect.adi_iterate_rect(G, BOX, p, q)
    assert _rel(Yd, Yc) < 1e-10
    # the J-step iterate meets the bound of Theorem 2.1 (the 2-norm error of
    # the iteration operator is at most the Zolotarev number bound)
    sx2, sy2 = rect.scalings(BOX)
    s = square.s_diag(n)
    Y = rect.solve_native_rect(G * np.outer(s, s), BOX) * np.outer(s, s)
    g = shifts.cross_ratio(*rect.rect_enclosure(n, BOX))
    err = np.linalg.norm(Y - Yc, 2) / np.linalg.norm(Y, 2)
    assert err <= shifts.zolotarev_bound(g, J) <= 1e-9


def test_rect_shifts_lie_in_their_intervals():
    n = 64
    a, b, c, d = rect.rect_enclosure(n, BOX)
    J, p, q = rect.rect_shifts(n, BOX, 1e-13)
    assert np.all((p >= a) & (p <= b))
    assert np.all((q >= c) & (q <= d))
    # the unequal scalings break the p = -q symmetry of the square
    assert np.abs(p + q).max() > 1e-3 * np.abs(p).max()


def test_coons_coefficients_match_sampled_interpolant():
    for n, seed in ((1, 1), (6, 2), (30, 3)):
        _, bc = workloads.rect_dirichlet_case(n, seed=seed)
        assert np.abs(rect.coons_coeffs(bc) - rect.coons_coeffs_sampled(bc)).max() < 1e-14
    # traces with trailing zeros: the sampled version uses a small grid
    n = 20
    _, small = workloads.rect_dirichlet_case(6, seed=2)
    bc = np.zeros((4, n + 2))
    bc[:, :8] = small
    assert np.abs(rect.coons_coeffs(bc) - rect.coons_coeffs_sampled(bc)).max() < 1e-14


def test_closed_form_ct_map():
    # against the Gauss-Jacobi quadrature map (absolute accuracy)
    for n in (1, 5, 40, 200):
        Rq = rect.cheb_to_ct_rect(n, n + 2)
        Rc = rect.cheb_to_ct_closed(n, n + 2)
        assert np.abs(Rq - Rc).max() < 1e-13
    # entrywise relative accuracy through the three-term recurrences:
    # x T_k = (T_{k+1} + T_{k-1})/2 and x C~_i = b_i C~_{i+1} + b_{i-1} C~_{i-1}
    # (b_i = sqrt((i+1)(i+3)/((2i+3)(2i+5))), the C~ Jacobi matrix)
    n = 1024
    Rc = rect.cheb_to_ct_closed(n + 1, n + 2)
    i = np.arange(n + 1, dtype=np.float64)
    b = np.sqrt((i + 1) * (i + 3) / ((2 * i + 3) * (2 * i + 5)))
    worst = 0.0
    for k in range(1, n + 1):
        c = Rc[:, k]
        xc = np.zeros(n + 1)
        xc[1:] += b[:-1] * c[:-1]
        xc[:-1] += b[:-1] * c[1:]
        rhs = 0.5 * (Rc[:, k + 1] + Rc[:, k - 1])
        sc = np.zeros(n + 1)
        sc[1:] += np.abs(b[:-1] * c[:-1])
        sc[:-1] += np.abs(b[:-1] * c[1:])
        sc += 0.5 * (np.abs(Rc[:, k + 1]) + np.abs(Rc[:, k - 1]))
        m = sc[:n] > 0
        worst = max(worst, float((np.abs(xc - rhs)[:n][m] / sc[:n][m]).max()))
    assert worst < 1e-13
    assert np.abs(Rc[Rc != 0]).min() < 1e-10  # tiny entries are resolved too


def test_lift_correction_is_confined_to_two_rows_and_columns():
    # Lap u_bc = sx2 [(1-t)/2 B'' + (1+t)/2 T''] + sy2 [(1-s)/2 L'' + (1+s)/2 R'']:
    # its C~ coefficients vanish off rows 0, 1 and columns 0, 1
    n = 512
    _, bc = workloads.rect_dirichlet_case(n, seed=5)
    C = rect.ct_projection(rect.laplacian_coeffs(rect.coons_coeffs(bc), BOX), n)
    assert np.abs(C[2:, 2:]).max() == 0.0
    assert np.abs(C[:2, :]).max() > 1.0


def test_second_derivative_recurrence_matches_numpy():
    g = workloads.decayed_normal(np.random.default_rng(1), (41,), 2.0)
    from numpy.polynomial import chebyshev as npc
    assert np.abs(rect.cheb_second_derivative(g) - npc.chebder(g, 2)).max() < 1e-13
    gl = rect.cheb_second_derivative(g.astype(np.longdouble))
    assert gl.dtype == np.longdouble


@pytest.mark.parametrize("n", [1, 2, 3, 30, 120])
def test_separable_lift_correction_matches_2d_definition(n):
    # the extended-precision separable form against the float64 projection of
    # the 2-D Chebyshev coefficients of Lap u_bc (smooth-enough traces at
    # these sizes for the latter to be accurate)
    _, bc = workloads.rect_dirichlet_case(n, seed=3)
    a = rect.lift_correction(bc, BOX, n)
    b = rect.lift_correction_2d(bc, BOX, n)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
