"""GPU parity of the square solver against the CPU oracle (through the C ABI)."""
import numpy as np
import pytest

import workloads
from oracle import shifts as oshifts, square

torch = pytest.importorskip("torch")
import paper_1710_11259_amd as fps  # noqa: E402

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.mark.parametrize("n,tol", [(1, 1e-13), (2, 1e-13), (5, 1e-13), (16, 1e-6), (64, 1e-13),
                                   (100, 1e-13), (257, 1e-10), (600, 1e-13), (1030, 1e-13)])
def test_adi_iterate_matches_closed_form(n, tol):
    # The J-step iterate of Algorithm 2 has a closed form for any shifts, so
    # this pins the sweeps independently of convergence.
    rng = np.random.default_rng(n)
    G = rng.standard_normal((n, n)) / np.outer(np.arange(1, n + 1), np.arange(1, n + 1))
    p = fps.plan(n, tol=tol)
    J, po, _ = oshifts.square_shifts(n, tol)
    assert p.J == J
    print(f"adi_native n={n} tol={tol} J={J}", flush=True)
    Y = fps.adi_native(p, _dev(G))
    torch.cuda.synchronize()
    Yo = square.adi_exact_iterate(G, po)
    assert _rel(Y.cpu().numpy(), Yo) < 1e-12


def test_long_chains_iterate_matches_closed_form():
    # n = 8200: 4100 positions per parity chain, i.e. 65 chunks, so each lane
    # of the chunk-carry scan owns 5 chunks, the last lane only one (a ragged
    # split).  The rounding of the J-step iterate grows with n (relative error
    # measured 1.7e-11 at n = 6000 and 1.2e-11 at n = 8192, 2.4e-11 here), so
    # the bound is 1e-10; a wrong carry gives errors of order one.
    n, tol = 8200, 1e-13
    rng = np.random.default_rng(n)
    G = rng.standard_normal((n, n)) / np.outer(np.arange(1, n + 1), np.arange(1, n + 1))
    p = fps.plan(n, tol=tol)
    J, po, _ = oshifts.square_shifts(n, tol)
    assert p.J == J
    print(f"adi_native n={n} J={J}", flush=True)
    Y = fps.adi_native(p, _dev(G)).cpu().numpy()
    print("closed form", flush=True)
    Yo = square.adi_exact_iterate(G, po)
    err = _rel(Y, Yo)
    print(f"rel err {err:.3e}", flush=True)
    assert err < 1e-10


@pytest.mark.parametrize("n", [1, 2, 3, 8, 64, 130, 513, 1024])
def test_solve_matches_exact_discrete_solution(n):
    F = workloads.square_rhs(n, seed=0)
    print(f"solve n={n}", flush=True)
    p = fps.plan(n, tol=1e-13)
    U = fps.solve(p, _dev(F))
    torch.cuda.synchronize()
    Uo = square.poisson_square(F)
    assert U.shape == (n + 2, n + 2)
    assert _rel(U.cpu().numpy(), Uo) <= 1e-12


@pytest.mark.parametrize("n", [7, 64, 300])
def test_native_output_matches(n):
    F = workloads.square_rhs(n, seed=3)
    p = fps.plan(n, tol=1e-13, out="native")
    X = fps.solve(p, _dev(F))
    torch.cuda.synchronize()
    Xo = square.poisson_square(F, out="native")
    assert _rel(X.cpu().numpy(), Xo) <= 1e-12


def test_manufactured_solution_accuracy():
    n = 64
    F, u_fun = workloads.manufactured_square(n, N=96)
    U = fps.solve(fps.plan(n, tol=1e-13), _dev(F))
    torch.cuda.synchronize()
    Uex = workloads.cheb_coeffs_2d(u_fun, n + 2)
    assert np.abs(U.cpu().numpy() - Uex).max() < 1e-12


def test_bitwise_deterministic_and_reusable_workspace():
    n = 700
    F = _dev(workloads.square_rhs(n, seed=5))
    p = fps.plan(n, tol=1e-13)
    ws = fps.workspace(p)
    U1 = fps.solve(p, F, ws=ws).clone()
    U2 = fps.solve(p, F, ws=ws)
    torch.cuda.synchronize()
    assert torch.equal(U1, U2)


def test_headline_size_full_parity():
    # n = 4096 (the benchmark workload): full comparison with the oracle.
    n = 4096
    F = workloads.square_rhs(n, seed=0)
    print("headline n=4096 solve", flush=True)
    p = fps.plan(n, tol=1e-13)
    U = fps.solve(p, _dev(F))
    torch.cuda.synchronize()
    Ug = U.cpu().numpy()
    print("headline oracle", flush=True)
    Uo = square.poisson_square(F)
    err = _rel(Ug, Uo)
    print(f"n=4096 rel err {err:.3e}", flush=True)
    assert err <= 1e-12


def test_largest_workload_size_full_parity():
    # n = 10^4 (10^8 dof): full comparison with the oracle (measured 6.6e-14).
    n = 10000
    F = workloads.square_rhs(n, seed=0)
    print("n=10000 solve", flush=True)
    p = fps.plan(n, tol=1e-13, tight=True)
    U = fps.solve(p, _dev(F)).cpu().numpy()
    print("n=10000 oracle", flush=True)
    Uo = square.poisson_square(F)
    err = _rel(U, Uo)
    print(f"n=10000 rel err {err:.3e}", flush=True)
    assert err <= 1e-12


@pytest.mark.parametrize("n", [1, 5, 64, 300, 1024, 4096])
def test_tight_spectrum_solve_matches_exact(n):
    # Shift intervals from the computed spectrum (fewer iterations, same bound).
    F = workloads.square_rhs(n, seed=0)
    p = fps.plan(n, tol=1e-13, tight=True)
    print(f"tight n={n} J={p.J}", flush=True)
    U = fps.solve(p, torch.from_numpy(F).cuda())
    torch.cuda.synchronize()
    Uo = square.poisson_square(F)
    err = np.linalg.norm(U.cpu().numpy() - Uo) / np.linalg.norm(Uo)
    print(f"rel err {err:.3e}", flush=True)
    assert err <= 1e-12
