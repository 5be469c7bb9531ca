"""ADI iteration count, Zolotarev shifts and error bounds.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper passages:
* Theorem 2.1, (2.4): p_j = T(-alpha dn[(2j+1)K(kappa)/(2J), kappa]),
  q_j = T(+alpha dn[...]), kappa = sqrt(1 - 1/alpha^2), alpha = -1 + 2 gamma
  + 2 sqrt(gamma^2 - gamma), gamma = |c-a||d-b| / (|c-b||d-a|), T the Moebius
  map sending {-alpha, -1, 1, alpha} to {a, b, c, d}.
* (2.5): Z_J <= 4 exp(pi^2 / (4 mu(1/sqrt(gamma))))^(-2J), with the Groetzsch
  ring function mu(lambda) = (pi/2) K(sqrt(1-lambda^2)) / K(lambda).
* (2.7): the same bound with 4 mu(1/sqrt gamma) replaced by 2 log(16 gamma).
* (2.9): J = ceil(log(16 gamma) log(4/eps) / pi^2).
* App. A: for alpha >= 1e7 the shifts are evaluated from the leading terms of
  the expansions of K and dn in the complementary parameter 1/alpha^2.
* App. B, (B.1): sigma(A~) in [-1, -1/(30 n^4)] for the square.

Elliptic functions here take the parameter m = kappa^2 (the App. A remark on
conventions); they are evaluated with mpmath at 60 significant digits.
"""
from __future__ import annotations

import math

import mpmath as mp
import numpy as np

_DPS = 60


def square_enclosure(n: int):
    """[a, b] = [-1, -1/(30 n^4)] for sigma(A~), [c, d] = [-b, -a] for
    sigma(B~) = sigma(-A~)  (Lemma B.1 and property P2 of Sec. 3.3)."""
    delta = 1.0 / (30.0 * float(n) ** 4)
    return -1.0, -delta, delta, 1.0


def cross_ratio(a, b, c, d):
    """gamma of Theorem 2.1."""
    return abs(c - a) * abs(d - b) / (abs(c - b) * abs(d - a))


def iteration_count(a, b, c, d, tol) -> int:
    """J of (2.9)."""
    if not (0.0 < tol < 1.0):
        raise ValueError("tol must lie in (0, 1)")
    g = cross_ratio(a, b, c, d)
    return int(math.ceil(math.log(16.0 * g) * math.log(4.0 / tol) / math.pi ** 2))


def clean_bound(gamma: float, J: int) -> float:
    """Right-hand side of (2.7): 4 exp(pi^2 / (2 log(16 gamma)))^(-2J)."""
    return 4.0 * math.exp(-2.0 * J * math.pi ** 2 / (2.0 * math.log(16.0 * gamma)))


def zolotarev_bound(gamma: float, J: int) -> float:
    """Right-hand side of (2.5) with the Groetzsch function evaluated exactly
    (moduli converted to parameters for mpmath's ellipk)."""
    with mp.workdps(_DPS):
        lam = 1 / mp.sqrt(mp.mpf(gamma))
        mu = mp.pi / 2 * mp.ellipk(1 - lam ** 2) / mp.ellipk(lam ** 2)
        return float(4 * mp.exp(-2 * J * mp.pi ** 2 / (4 * mu)))


def mobius_coefficients(a, b, c, d, alpha):
    """(A, B, C, D) with T(z) = (A z + B)/(C z + D) sending -alpha -> a,
    -1 -> b, 1 -> c.  Found as the null vector of the 3 x 4 linear system
    A z_i + B - w_i C z_i - w_i D = 0; T(alpha) = d follows from the equal
    cross-ratios (proof of Theorem 2.1) and is checked by the tests."""
    with mp.workdps(_DPS):
        z = [-mp.mpf(alpha), mp.mpf(-1), mp.mpf(1)]
        w = [mp.mpf(a), mp.mpf(b), mp.mpf(c)]
        Mx = mp.matrix([[z[i], 1, -w[i] * z[i], -w[i]] for i in range(3)])
        # null vector by fixing D = 1 when possible
        sub = mp.matrix([[Mx[i, 0], Mx[i, 1], Mx[i, 2]] for i in range(3)])
        rhs = mp.matrix([-Mx[i, 3] for i in range(3)])
        sol = mp.lu_solve(sub, rhs)
        return sol[0], sol[1], sol[2], mp.mpf(1)


def _alpha(gamma):
    with mp.workdps(_DPS):
        g = mp.mpf(gamma)
        return -1 + 2 * g + 2 * mp.sqrt(g * g - g)


def zolotarev_shifts(a, b, c, d, tol=None, J=None):
    """(J, p, q) of Theorem 2.1 with J from (2.9) unless given."""
    if J is None:
        J = iteration_count(a, b, c, d, tol)
    gamma = cross_ratio(a, b, c, d)
    with mp.workdps(_DPS):
        al = _alpha(gamma)
        m = 1 - 1 / al ** 2
        K = mp.ellipk(m)
        A, B, C, D = mobius_coefficients(a, b, c, d, al)
        T = lambda zz: (A * zz + B) / (C * zz + D)  # noqa: E731
        p, q = [], []
        for j in range(J):
            dn = mp.ellipfun("dn", (2 * j + 1) * K / (2 * J), m=m)
            p.append(float(T(-al * dn)))
            q.append(float(T(al * dn)))
    return J, np.array(p), np.array(q)


def square_shifts(n: int, tol: float):
    """Shifts for A~ Y - Y(-A~) = G on the enclosure of Lemma B.1."""
    return zolotarev_shifts(*square_enclosure(n), tol=tol)


def appendix_a_large_alpha_dn(alpha: float, J: int) -> np.ndarray:
    """dn((j+1/2) K / J) from the App. A large-alpha formulas, m1 = 1/alpha^2:
    K ~ 2 log 2 + log alpha + (-1 + 2 log 2 + log alpha) m1 / 4,
    dn(u) ~ sech u + (m1/4)(sinh u cosh u + u) tanh u sech u."""
    m1 = 1.0 / alpha ** 2
    K = (2 * math.log(2) + math.log(alpha)) + (-1 + 2 * math.log(2) + math.log(alpha)) * m1 / 4
    u = (np.arange(J) + 0.5) * K / J
    sech = 1.0 / np.cosh(u)
    return sech + 0.25 * m1 * (np.sinh(u) * np.cosh(u) + u) * np.tanh(u) * sech


def exact_dn(alpha: float, J: int) -> np.ndarray:
    """dn((j+1/2) K(m)/J | m), m = 1 - 1/alpha^2, at 60 digits."""
    with mp.workdps(_DPS):
        al = mp.mpf(alpha)
        m = 1 - 1 / al ** 2
        K = mp.ellipk(m)
        return np.array([float(mp.ellipfun("dn", (j + mp.mpf(1) / 2) * K / J, m=m))
                         for j in range(J)])


def rational_factor(lam: np.ndarray, p: np.ndarray, q: np.ndarray) -> np.ndarray:
    """r(z) = prod (z - p_j) / prod (z - q_j) of Sec. 2 (the P1 bound),
    evaluated as a product of ratios."""
    r = np.ones_like(lam, dtype=np.float64)
    for pj, qj in zip(p, q):
        r *= (lam - pj) / (lam - qj)
    return r
