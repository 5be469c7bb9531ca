"""Pins for oracle.shifts: Moebius map, elliptic-function identities, the
App. A large-alpha branch, (2.9) against (2.7), and the P1 error bound."""
import math

import numpy as np
import pytest

from oracle import shifts


@pytest.mark.parametrize("iv", [(-1.0, -1e-3, 1e-3, 1.0), (-5.0, -0.5, 0.2, 3.0), (-4.0, -1.0, 1.0, 4.0)])
def test_mobius_maps_all_four_points(iv):
    a, b, c, d = iv
    g = shifts.cross_ratio(a, b, c, d)
    al = float(shifts._alpha(g))
    A, B, C, D = shifts.mobius_coefficients(a, b, c, d, al)
    T = lambda z: float((A * z + B) / (C * z + D))  # noqa: E731
    for z, w in zip((-al, -1.0, 1.0, al), iv):
        assert abs(T(z) - w) < 1e-12 * max(1.0, abs(w))


def test_symmetric_enclosure_gives_linear_map_and_alpha():
    # [a,b] = [-1,-delta], [c,d] = [delta,1]: alpha = 1/delta, T(z) = delta z
    n = 16
    a, b, c, d = shifts.square_enclosure(n)
    delta = -b
    g = shifts.cross_ratio(a, b, c, d)
    al = float(shifts._alpha(g))
    assert abs(al * delta - 1) < 1e-12
    J, p, q = shifts.square_shifts(n, 1e-13)
    dn = shifts.exact_dn(al, J)
    assert np.allclose(p, -delta * al * dn, rtol=1e-14)
    assert np.allclose(q, -p, rtol=1e-14)


@pytest.mark.parametrize("n", [4, 64, 1024])
def test_shift_pairs_multiply_to_delta(n):
    # dn(K-u) = k'/dn(u) with k' = 1/alpha, and u_{J-1-j} = K - u_j,
    # so p_j p_{J-1-j} = delta in the symmetric case.
    J, p, _ = shifts.square_shifts(n, 1e-13)
    delta = 1.0 / (30.0 * n ** 4)
    assert np.allclose(p * p[::-1], delta, rtol=1e-12)
    assert np.all(p < 0) and np.all(np.diff(p) > 0)  # increasing toward -delta


@pytest.mark.parametrize("n", [32, 64, 256, 4096])
def test_appendix_a_branch_matches_exact_dn(n):
    alpha = 30.0 * n ** 4
    assert alpha >= 1e7
    J = shifts.iteration_count(*shifts.square_enclosure(n), 1e-13)
    approx = shifts.appendix_a_large_alpha_dn(alpha, J)
    exact = shifts.exact_dn(alpha, J)
    assert np.max(np.abs(approx / exact - 1)) < 1e-13


@pytest.mark.parametrize("tol", [1e-3, 1e-8, 1e-13])
@pytest.mark.parametrize("n", [8, 64, 4096, 10000])
def test_iteration_count_is_least_J_meeting_bound_2_7(n, tol):
    a, b, c, d = shifts.square_enclosure(n)
    g = shifts.cross_ratio(a, b, c, d)
    J = shifts.iteration_count(a, b, c, d, tol)
    assert shifts.clean_bound(g, J) <= tol * (1 + 1e-12)
    assert shifts.clean_bound(g, J - 1) > tol


def test_known_square_counts():
    # (2.9) for the workload sizes at tol 1e-13 (worked from the formula by hand:
    # log(16 gamma) ~ log(120 n^4), log(4/eps) = 31.32)
    counts = {n: shifts.iteration_count(*shifts.square_enclosure(n), 1e-13)
              for n in (64, 1024, 2048, 4096, 10000)}
    assert counts == {64: 68, 1024: 104, 2048: 112, 4096: 121, 10000: 133}


def test_bound_2_5_below_2_7():
    for n in (8, 100, 4096):
        g = shifts.cross_ratio(*shifts.square_enclosure(n))
        for J in (5, 20, 60):
            assert shifts.zolotarev_bound(g, J) <= shifts.clean_bound(g, J) * (1 + 1e-12)


def test_zolotarev_error_factor_within_bound_on_interval():
    # sup_{[a,b]} |r| / inf_{[c,d]} |r| <= Z_J bound (2.5), sampled densely
    n, tol = 16, 1e-10
    a, b, c, d = shifts.square_enclosure(n)
    J, p, q = shifts.square_shifts(n, tol)
    z1 = -np.geomspace(-b, -a, 20001)
    z2 = np.geomspace(c, d, 20001)
    ratio = np.abs(shifts.rational_factor(z1, p, q)).max() / np.abs(shifts.rational_factor(z2, p, q)).min()
    g = shifts.cross_ratio(a, b, c, d)
    assert ratio <= shifts.zolotarev_bound(g, J) * (1 + 1e-9)
    assert ratio <= tol


def test_tol_validation():
    with pytest.raises(ValueError):
        shifts.iteration_count(-1, -0.1, 0.1, 1, 1.5)
