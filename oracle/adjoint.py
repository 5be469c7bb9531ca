"""Adjoint (vector-Jacobian product) of the square solve F_T -> U.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The solve is the composition of explicit linear maps (Sec. 3.4 and Table 1):
    F_C = R F_T R^T,  G = S^-1 F_C S^-1,  Y = L^-1 G  (L Y = A~ Y + Y A~),
    X = S^-1 Y S^-1,  U = P X P^T,
so its adjoint in the Frobenius inner product is the composition of the
transposes in reverse order.  L is self-adjoint because A~ is symmetric.
"""
from __future__ import annotations

import numpy as np

from . import basis
from .square import s_diag, solve_symmetric_sylvester, adi_exact_iterate


def vjp_square(Ubar: np.ndarray, p=None) -> np.ndarray:
    """F_T-bar for the exact solve (p None) or for the J-step ADI map with
    shifts p.  Ubar is (n+2) x (n+2); the result is n x n."""
    n = Ubar.shape[0] - 2
    P = basis.recombined_to_cheb(n)
    R = basis.cheb_to_ct(n)
    s = s_diag(n)
    Xbar = P.T @ Ubar @ P
    Ybar = Xbar / np.outer(s, s)
    if p is None:
        Gbar = solve_symmetric_sylvester(Ybar)
    else:
        Gbar = adi_exact_iterate(Ybar, p)
    FCbar = Gbar / np.outer(s, s)
    return R.T @ FCbar @ R
