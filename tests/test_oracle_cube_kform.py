"""Pins of the oracle's two-level (K-form) nested ADI for the cube against
the exact eigen-decomposition solution (itself pinned against a brute-force
Kronecker solve), the closed form of the outer iterate, the Zolotarev bound
of Theorem 2.1 and the spectral enclosure of Lemma B.1."""
import numpy as np
import pytest

import workloads
from oracle import cube, shifts, square


def _case(n, seed=2):
    F = workloads.cube_rhs(n, seed=seed)
    FC = cube.rhs_ct(F)
    G = cube.symmetric_rhs(FC)
    s = square.s_diag(n)
    Y = cube.solve_native(FC) * s[:, None, None] * s[None, :, None] * s[None, None, :]
    return G, Y


@pytest.mark.parametrize("n", [1, 3, 8])
def test_kform_identity_holds_for_exact_solution(n):
    # (K_x + K_y + K_z) Y = (A~^-1)^{x3} G with K = -A~^-1.
    G, Y = _case(n)
    Ai = np.linalg.inv(square.atilde_dense(n))
    lhs = sum(cube.mode_product(Y, -Ai, m) for m in range(3))
    B = cube.kform_rhs(G)
    assert np.linalg.norm(lhs - B) <= 1e-13 * np.linalg.norm(B)


@pytest.mark.parametrize("n", [2, 6])
def test_outer_iterate_with_exact_inner_matches_closed_form(n):
    G, _ = _case(n)
    Y, J, _ = cube.kform_adi(G, 1e-9, 1e-14, inner_exact=True)
    Yc = cube.kform_outer_closed_form(G, 1e-9)
    assert np.linalg.norm(Y - Yc) <= 1e-13 * np.linalg.norm(Yc)


@pytest.mark.parametrize("n,tol", [(4, 1e-6), (10, 1e-10), (16, 1e-13)])
def test_outer_error_factor_within_zolotarev_bound(n, tol):
    # max over eigen-triples of |r| <= the Theorem 2.1 bound for the outer
    # intervals; a wrong interval (e.g. sigma(H) taken as [1, 1/delta])
    # breaks this at small n.
    lam, _ = square.atilde_eig(n)
    kap = -1.0 / lam
    J, p, q = cube.kform_outer_shifts(n, tol)
    a = -(kap[:, None] + kap[None, :]).reshape(-1)[:, None]
    b = kap[None, :]
    r = np.ones(np.broadcast(a, b).shape)
    for pj, qj in zip(p, q):
        r = r * ((a - pj) * (b - qj)) / ((a - qj) * (b - pj))
    delta = 1.0 / (30.0 * n ** 4)
    gamma = shifts.cross_ratio(-2 / delta, -2.0, 1.0, 1 / delta)
    assert np.max(np.abs(r)) <= shifts.zolotarev_bound(gamma, J) * (1 + 1e-9)
    assert shifts.zolotarev_bound(gamma, J) <= tol


def test_kform_spectra_inside_enclosures():
    n = 20
    lam, _ = square.atilde_eig(n)
    kap = -1.0 / lam
    delta = 1.0 / (30.0 * n ** 4)
    assert kap.min() >= 1.0 and kap.max() <= 1.0 / delta


@pytest.mark.parametrize("n", [1, 4, 9])
def test_nested_kform_adi_matches_exact_solution(n):
    G, Y = _case(n)
    Yk, J1, J2 = cube.kform_adi(G, 1e-13, 1e-14)
    s = square.s_diag(n)
    w = 1.0 / (s[:, None, None] * s[None, :, None] * s[None, None, :])
    err = np.linalg.norm((Yk - Y) * w) / np.linalg.norm(Y * w)
    assert err <= 1e-12
    assert len(J2) == J1 and min(J2) >= 1


@pytest.mark.parametrize("n", [1, 4, 9])
@pytest.mark.parametrize("tight", [True, False])
def test_zeig_slice_adi_matches_exact_solution(n, tight):
    G, Y = _case(n)
    Yz, counts = cube.zeig_adi(G, 1e-13, tight=tight)
    s = square.s_diag(n)
    w = 1.0 / (s[:, None, None] * s[None, :, None] * s[None, None, :])
    err = np.linalg.norm((Yz - Y) * w) / np.linalg.norm(Y * w)
    assert err <= 1e-12
    assert len(counts) == n


def test_zeig_slice_intervals_contain_spectra():
    # sigma(-mu^2 P^-1) and sigma(-P) inside the stated intervals, which are
    # separated by |mu|.
    n = 24
    A = square.atilde_dense(n)
    lam, _ = square.atilde_eig(n)
    for mu in lam[:: 5]:
        P = A + mu * np.eye(n)
        ea = np.linalg.eigvalsh(-mu * mu * np.linalg.inv(P))
        eb = np.linalg.eigvalsh(-P)
        a, b, c, d = cube.zeig_slice_intervals(n, mu, lam.min(), lam.max())
        assert a * (1 - 1e-12) <= ea.min() and ea.max() <= b * (1 + 1e-12)
        assert c * (1 - 1e-12) <= eb.min() and eb.max() <= d * (1 + 1e-12)
        assert b < abs(mu) < c
