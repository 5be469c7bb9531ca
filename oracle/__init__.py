"""CPU FP64 oracle for the spectral Poisson solver of Fortunato & Townsend,
"Fast Poisson solvers for spectral methods" (arXiv 1710.11259).

TEST INFRASTRUCTURE ONLY.  This package is the independent reference the HIP
solver is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code,
tables or constants with the product library: it is written with NumPy,
SciPy (LAPACK/BLAS) and mpmath, in float64 unless stated, and follows the
paper's definitions as plainly as possible:

* ``basis``   -- the normalized ultraspherical basis C~^(3/2) (Sec. 3.1,
                 footnote on normalization), the multiplication matrix M of
                 (3.7), the diagonal D of (3.6), and the coefficient maps
                 Chebyshev <-> C~ by Gauss-Jacobi quadrature and by
                 evaluation on a Chebyshev grid plus a discrete cosine sum.
* ``shifts``  -- the spectral enclosure of App. B (B.1), the iteration count
                 (2.9), the Zolotarev shifts of Theorem 2.1 (2.4) evaluated
                 with 60-digit elliptic functions, the large-alpha formulas
                 of App. A, and the bounds (2.5) and (2.7).
* ``square``  -- the exact solution of the discrete system (3.6) (symmetrized
                 as in (3.9), with the similarity transform read as a
                 congruence) by eigendecomposition, a brute-force Kronecker
                 solve for tiny n, Algorithm 2 written out with dense solves,
                 the closed form of its J-th iterate, and the whole square
                 pipeline F_T -> X -> U.
* ``cube``    -- the exact solution of the cube system (5.2) (with the
                 right-hand side scaled by D^-1 in each mode) and a
                 brute-force Kronecker solve.
* ``rect``    -- the rectangle [a,b] x [c,d] (scaled operators on the two
                 sides, general-interval shifts of Theorem 2.1, the closed
                 form of Algorithm 2's iterate) and nonhomogeneous Dirichlet
                 data by a transfinite lift (Sec. 6.1).
* ``cylinder`` -- the cylinder (Sec. 4.1): DFS-doubled Chebyshev-Fourier-
                 Chebyshev data, one Galerkin system per Fourier mode (three
                 cases of partial regularity), Bartels-Stewart or Kronecker.
* ``adjoint`` -- the transpose of the whole linear map F_T -> U.
* ``fd``      -- the five-point finite-difference Sylvester equation (1.2)
                 and its sine-transform solution (1.3), used to check the
                 shift machinery on a textbook problem.

Where the paper is ambiguous or in error, the oracle takes these readings:
the iteration count (2.9) rather than the square-case display of Sec. 3.3;
the congruence in (3.9); the rectangular M on output; the cube right-hand
side scaled by D^-1 in each mode; and the further readings stated in the
docstrings of the rect and cylinder modules.
"""
from . import basis, shifts, square, cube, adjoint, fd, rect, cylinder  # noqa: F401
