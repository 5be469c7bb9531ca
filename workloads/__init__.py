"""Seeded synthetic inputs for the spectral Poisson solver.

This module is shared by the oracle, the tests and the benchmark.  It holds
no arithmetic of the solver itself: it only draws seeded random coefficient
arrays with the decay profiles of the workloads, and samples the manufactured
right-hand sides (analytic Laplacians of closed-form solutions) on Chebyshev
grids.

Conventions (rows <-> y, columns <-> x, as in the expansion (3.2)):
  square: F[j, k] is the coefficient of T_j(y) T_k(x);
  cube:   F[i, j, k] is the coefficient of T_i(z) T_j(y) T_k(x).
All arrays are float64, C-contiguous.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "decayed_normal", "square_rhs", "cube_rhs", "batched_problems",
    "adjoint_case", "cheb_coeffs_2d", "cheb_coeffs_3d",
    "manufactured_square", "manufactured_cube", "oscillatory_square_rhs",
    "rect_dirichlet_case", "manufactured_rect", "cylinder_rhs", "cylinder_coeffs",
    "manufactured_cylinder",
]


def decayed_normal(rng: np.random.Generator, shape, decay: float) -> np.ndarray:
    """N(0,1) entries drawn in C order, multiplied by prod_axis (1+idx)^-decay."""
    F = rng.standard_normal(shape)
    for ax, n in enumerate(shape):
        w = (1.0 + np.arange(n, dtype=np.float64)) ** (-decay)
        sh = [1] * len(shape)
        sh[ax] = n
        F *= w.reshape(sh)
    return np.ascontiguousarray(F)


def square_rhs(n: int, seed: int = 0, decay: float = 2.0) -> np.ndarray:
    """F_jk = N(0,1) (1+j)^-decay (1+k)^-decay, default_rng(seed)."""
    return decayed_normal(np.random.default_rng(seed), (n, n), decay)


def cube_rhs(n: int, seed: int = 2, decay: float = 2.0) -> np.ndarray:
    """F_ijk = N(0,1) (1+i)^-2 (1+j)^-2 (1+k)^-2, default_rng(seed)."""
    return decayed_normal(np.random.default_rng(seed), (n, n, n), decay)


def batched_problems(count: int = 256, seed: int = 1, step: int = 32,
                     nmax_steps: int = 32, decay: float = 1.5):
    """Sizes n_b = step * U{1..nmax_steps} then each F_b, all from one rng."""
    rng = np.random.default_rng(seed)
    sizes = [int(s) for s in step * rng.integers(1, nmax_steps + 1, count)]
    Fs = [decayed_normal(rng, (n, n), decay) for n in sizes]
    return sizes, Fs


def adjoint_case(n: int, batch: int, n_dirs: int = 32, seed_f: int = 0,
                 seed_target: int = 3, seed_dirs: int = 4):
    """Differentiable-solve workload: inputs F (batch, n, n), target right-hand
    side F* (seed 3) and unit-Frobenius Gaussian directions (seed 4)."""
    rng = np.random.default_rng(seed_f)
    F = np.stack([decayed_normal(rng, (n, n), 2.0) for _ in range(batch)])
    Fstar = decayed_normal(np.random.default_rng(seed_target), (n, n), 2.0)
    rd = np.random.default_rng(seed_dirs)
    dirs = rd.standard_normal((n_dirs, batch, n, n))
    dirs /= np.sqrt((dirs ** 2).sum(axis=(1, 2, 3), keepdims=True))
    return F, Fstar, dirs


# --- Chebyshev interpolation of sampled functions (input preparation) -------

def _cheb_points(N: int) -> np.ndarray:
    # first-kind points x_m = cos((m + 1/2) pi / N)
    return np.cos((np.arange(N) + 0.5) * np.pi / N)


def _dct_coeffs_axis(vals: np.ndarray, axis: int) -> np.ndarray:
    N = vals.shape[axis]
    m = np.arange(N)
    C = np.cos(np.outer(np.arange(N), (m + 0.5) * np.pi / N)) * (2.0 / N)
    C[0] *= 0.5
    return np.moveaxis(np.tensordot(C, vals, axes=([1], [axis])), 0, axis)


def cheb_coeffs_2d(fun, N: int) -> np.ndarray:
    """Chebyshev coefficients C[j, k] (T_j(y) T_k(x)) of the degree-(N-1)
    interpolant of fun(x, y) on the N x N first-kind grid."""
    x = _cheb_points(N)
    Y, X = np.meshgrid(x, x, indexing="ij")
    v = fun(X, Y)
    return _dct_coeffs_axis(_dct_coeffs_axis(v, 0), 1)


def cheb_coeffs_3d(fun, N: int) -> np.ndarray:
    x = _cheb_points(N)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    v = fun(X, Y, Z)
    for ax in range(3):
        v = _dct_coeffs_axis(v, ax)
    return v


def _pad(C: np.ndarray, n: int) -> np.ndarray:
    out = np.zeros((n,) * C.ndim)
    sl = tuple(slice(0, min(n, s)) for s in C.shape)
    out[sl] = C[sl]
    return out


def manufactured_square(n: int, N: int = 128):
    """u = (1-x^2)(1-y^2) exp(sin 3x cos 2y) and f = Lap u.

    Returns (F, u_fun): F are the n x n Chebyshev coefficients of f (the
    degree-(N-1) interpolant, truncated or zero-padded to n), u_fun(x, y)
    evaluates the exact solution."""
    def u_fun(x, y):
        return (1 - x * x) * (1 - y * y) * np.exp(np.sin(3 * x) * np.cos(2 * y))

    def f_fun(x, y):
        a, b = 1 - x * x, 1 - y * y
        s = np.sin(3 * x) * np.cos(2 * y)
        E = np.exp(s)
        sx = 3 * np.cos(3 * x) * np.cos(2 * y)
        sxx = -9 * np.sin(3 * x) * np.cos(2 * y)
        sy = -2 * np.sin(3 * x) * np.sin(2 * y)
        syy = -4 * np.sin(3 * x) * np.cos(2 * y)
        uxx = b * E * (-2 + 2 * (-2 * x) * sx + a * (sx * sx + sxx))
        uyy = a * E * (-2 + 2 * (-2 * y) * sy + b * (sy * sy + syy))
        return uxx + uyy

    return _pad(cheb_coeffs_2d(f_fun, N), n), u_fun


def manufactured_cube(n: int, N: int = 48):
    """u = (1-x^2)(1-y^2)(1-z^2) cos(x y z^2) and f = Lap u (Fig. cube)."""
    def u_fun(x, y, z):
        return (1 - x * x) * (1 - y * y) * (1 - z * z) * np.cos(x * y * z * z)

    def f_fun(x, y, z):
        a, b, c = 1 - x * x, 1 - y * y, 1 - z * z
        t = x * y * z * z
        C, S = np.cos(t), np.sin(t)
        tx, txx = y * z * z, 0.0
        ty, tyy = x * z * z, 0.0
        tz, tzz = 2 * x * y * z, 2 * x * y
        # g = cos(t): g' = -S t', g'' = -C t'^2 - S t''
        gx, gxx = -S * tx, -C * tx * tx - S * txx
        gy, gyy = -S * ty, -C * ty * ty - S * tyy
        gz, gzz = -S * tz, -C * tz * tz - S * tzz
        uxx = b * c * (-2 * C + 2 * (-2 * x) * gx + a * gxx)
        uyy = a * c * (-2 * C + 2 * (-2 * y) * gy + b * gyy)
        uzz = a * b * (-2 * C + 2 * (-2 * z) * gz + c * gzz)
        return uxx + uyy + uzz

    return _pad(cheb_coeffs_3d(f_fun, N), n), u_fun


def oscillatory_square_rhs(n: int, N: int = 256) -> np.ndarray:
    """f = -100 x sin(20 pi x^2 y) cos(4 pi (x + y)) (Fig. square, left)."""
    def f_fun(x, y):
        return -100 * x * np.sin(20 * np.pi * x * x * y) * np.cos(4 * np.pi * (x + y))
    return _pad(cheb_coeffs_2d(f_fun, N), n)


# --- Rectangle with Dirichlet data -------------------------------------------
#
# Boundary data are four Chebyshev series of length n + 2 in the mapped
# variables s = (2x - a - b)/(b - a), t = (2y - c - d)/(d - c):
#   L(t) = u(a, y), R(t) = u(b, y), B(s) = u(x, c), T(s) = u(x, d),
# stored as the rows of one (4, n + 2) array in that order.

def _cheb_coeffs_1d(vals: np.ndarray) -> np.ndarray:
    return _dct_coeffs_axis(vals, 0)


def _line_fix(v: np.ndarray, lo: float, hi: float) -> np.ndarray:
    # add alpha T_0 + beta T_1 so that the series takes lo at -1 and hi at +1
    k = np.arange(v.size)
    at_m1 = float(((-1.0) ** k) @ v)
    at_p1 = float(v.sum())
    out = v.copy()
    out[0] += ((lo - at_m1) + (hi - at_p1)) / 2
    out[1] += ((hi - at_p1) - (lo - at_m1)) / 2
    return out


def rect_dirichlet_case(n: int, seed: int = 5, decay: float = 2.0):
    """(F, bc): random right-hand side as for the square, and four random
    traces (decayed normal, seed+1) with L and R adjusted in their two
    leading coefficients so that the four corners agree."""
    F = decayed_normal(np.random.default_rng(seed), (n, n), decay)
    rng = np.random.default_rng(seed + 1)
    L, R, B, T = (decayed_normal(rng, (n + 2,), decay) for _ in range(4))
    k = np.arange(n + 2)
    B_m1, B_p1 = float(((-1.0) ** k) @ B), float(B.sum())
    T_m1, T_p1 = float(((-1.0) ** k) @ T), float(T.sum())
    L = _line_fix(L, B_m1, T_m1)  # L(-1) = u(a, c) = B(-1), L(1) = u(a, d) = T(-1)
    R = _line_fix(R, B_p1, T_p1)  # R(-1) = u(b, c) = B(1),  R(1) = u(b, d) = T(1)
    return F, np.ascontiguousarray(np.stack([L, R, B, T]))


def manufactured_rect(n: int, box, N: int = 96):
    """u = exp(x/2) cos(3y/2) + sin(x y) on the box (a, b, c, d), f = Lap u =
    -2 exp(x/2) cos(3y/2) - (x^2 + y^2) sin(x y).

    Returns (F, bc, u_fun): F the n x n Chebyshev coefficients of f in the
    mapped variables, bc the (4, n + 2) boundary traces (interpolants on N
    points, truncated), u_fun(s, t) the exact solution in mapped variables."""
    a, b, c, d = box

    def xs(s):
        return (a + b) / 2 + (b - a) / 2 * s

    def yt(t):
        return (c + d) / 2 + (d - c) / 2 * t

    def u_fun(s, t):
        x, y = xs(s), yt(t)
        return np.exp(x / 2) * np.cos(1.5 * y) + np.sin(x * y)

    def f_fun(s, t):
        x, y = xs(s), yt(t)
        return -2 * np.exp(x / 2) * np.cos(1.5 * y) - (x * x + y * y) * np.sin(x * y)

    F = _pad(cheb_coeffs_2d(f_fun, N), n)
    p = _cheb_points(N)
    one = np.ones(N)
    traces = [u_fun(-one, p), u_fun(one, p), u_fun(p, -one), u_fun(p, one)]
    bc = np.stack([_pad(_cheb_coeffs_1d(v), n + 2) for v in traces])
    return F, np.ascontiguousarray(bc), u_fun


# --- Cylinder (DFS doubling, Chebyshev(r) x Fourier(theta) x Chebyshev(z)) ---
#
# Arrays F[idx, i, j], idx = k + n_theta/2 for Fourier modes
# k = -n_theta/2 .. n_theta/2 - 1, i <-> T_i(r) on the doubled r in [-1, 1],
# j <-> T_j(z); complex128.

def cylinder_rhs(n: int, n_theta: int, seed: int = 7, decay: float = 2.0) -> np.ndarray:
    """Random doubled-up right-hand side: real and imaginary parts N(0,1)
    (1+i)^-decay (1+j)^-decay (1+|k|)^-decay, with the r-parity of a doubled
    function (mode k has only coefficients i = k mod 2)."""
    rng = np.random.default_rng(seed)
    F = decayed_normal(rng, (n_theta, n, n), decay) + 1j * decayed_normal(rng, (n_theta, n, n), decay)
    ks = np.arange(n_theta) - n_theta // 2
    w = (1.0 + np.abs(ks)) ** (-decay)
    i = np.arange(n)
    mask = (i[None, :] % 2) == (np.abs(ks)[:, None] % 2)
    F *= (w[:, None] * mask)[:, :, None]
    return np.ascontiguousarray(F)


def cylinder_coeffs(fun, n: int, n_theta: int, N: int) -> np.ndarray:
    """Chebyshev-Fourier-Chebyshev coefficients (n_theta, n, n) of the
    doubled-up f~(r, theta, z) = fun(r cos theta, r sin theta, z): sampled on
    N first-kind points in r and z and n_theta points theta_l = -pi + 2 pi
    l / n_theta, transformed by the discrete cosine map and the FFT
    (f~_k = (1/n_theta) sum_l f~(theta_l) e^{-i k theta_l})."""
    r = _cheb_points(N)
    th = -np.pi + 2 * np.pi * np.arange(n_theta) / n_theta
    R, TH, Z = np.meshgrid(r, th, r, indexing="ij")  # [r, theta, z]
    v = fun(R * np.cos(TH), R * np.sin(TH), Z)
    v = _dct_coeffs_axis(_dct_coeffs_axis(v, 0), 2)
    ks = np.arange(n_theta) - n_theta // 2
    E = np.exp(-1j * np.outer(ks, th)) / n_theta  # [k, l]
    C = np.einsum("kl,ilj->kij", E, v)
    out = np.zeros((n_theta, n, n), dtype=np.complex128)
    m = min(n, N)
    out[:, :m, :m] = C[:, :m, :m]
    return out


def manufactured_cylinder(n: int, n_theta: int, N: int = 64):
    """u = (1 - x^2 - y^2)(1 - z^2)(z cos x^2 + cos yz) on the unit cylinder
    (the paper's cylinder example with the frequencies lowered), f = Lap u
    written out.  Returns (F, u_fun)."""
    def u_fun(x, y, z):
        return (1 - x * x - y * y) * (1 - z * z) * (z * np.cos(x * x) + np.cos(y * z))

    def f_fun(x, y, z):
        x2, y2, z2 = x * x, y * y, z * z
        return ((-4 * x2 * y * z - 4 * y ** 3 * z - 4 * y * z ** 3 + 8 * y * z) * np.sin(y * z)
                + (-10 * x2 * z ** 3 + 10 * x2 * z - 2 * y2 * z ** 3 + 2 * y2 * z + 2 * z ** 3 - 2 * z)
                * np.sin(x2)
                + (-4 * x2 * x2 * z ** 3 + 4 * x2 * x2 * z - 4 * x2 * y2 * z ** 3 + 4 * x2 * y2 * z
                   + 4 * x2 * z ** 3 + 2 * x2 * z + 6 * y2 * z + 4 * z ** 3 - 10 * z) * np.cos(x2)
                + (-x2 * y2 * z2 + x2 * y2 - x2 * z2 * z2 + x2 * z2 + 2 * x2 - y2 * y2 * z2 + y2 * y2
                   - y2 * z2 * z2 + 2 * y2 * z2 + y2 + z2 * z2 + 3 * z2 - 6) * np.cos(y * z))

    return cylinder_coeffs(f_fun, n, n_theta, N), u_fun, f_fun
