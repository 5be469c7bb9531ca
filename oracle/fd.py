"""Five-point finite-difference Poisson problem (1.2) and its fast
sine-transform solution (1.3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

(1.2): K X + X K^T = F, K = -(1/h^2) tridiag(-1, 2, -1) of size n-1, h = 2/n.
(1.3): X = S (C o (S^-1 F S^-T)) S^T, C_jk = 1/(lam_j + lam_k), with S the
normalized DST-I matrix and lam_k = -4/h^2 sin^2(pi k/(2n)).
Sec. 2.1, P2: sigma(K) in [-n^2, -1], sigma(-K^T) in [1, n^2].
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft


def K_matrix(n: int) -> np.ndarray:
    h = 2.0 / n
    m = n - 1
    K = (np.diag(np.full(m, 2.0)) - np.diag(np.ones(m - 1), 1)
         - np.diag(np.ones(m - 1), -1))
    return -K / h ** 2


def dst_solve(F: np.ndarray) -> np.ndarray:
    """(1.3) with the orthonormal DST-I (S = S^T = S^-1)."""
    n = F.shape[0] + 1
    h = 2.0 / n
    k = np.arange(1, n)
    lam = -4.0 / h ** 2 * np.sin(np.pi * k / (2 * n)) ** 2
    Fh = sfft.dstn(F, type=1, norm="ortho")
    return sfft.idstn(Fh / (lam[:, None] + lam[None, :]), type=1, norm="ortho")


def enclosure(n: int):
    return -float(n) ** 2, -1.0, 1.0, float(n) ** 2
