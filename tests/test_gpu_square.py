"""GPU parity of the square solver against the CPU oracle (through the C ABI)."""
import numpy as np
import pytest

import parity
import workloads
from oracle import shifts as oshifts, square

torch = pytest.importorskip("torch")
import paper_1710_11259_amd as fps  # noqa: E402

pytestmark = pytest.mark.gpu


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
    parity.check(Y.cpu().numpy(), Yo, 1e-12, f"adi_native n={n}")


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
    parity.check(Y, Yo, 1e-10, f"adi_native n={n}")


def test_mid_length_chains_iterate_matches_closed_form():
    # n = 6000: 3000 positions per parity chain, 47 chunks, so each lane of
    # the chunk-carry scan owns 3 chunks (the scan form for 33 to 64 chunks
    # per chain); the bound follows the rounding of the iterate at this n
    # (measured 1.7e-11), a wrong carry gives errors of order one.
    n, tol = 6000, 1e-13
    rng = np.random.default_rng(n)
    G = rng.standard_normal((n, n)) / np.outer(np.arange(1, n + 1), np.arange(1, n + 1))
    p = fps.plan(n, tol=tol)
    J, po, _ = oshifts.square_shifts(n, tol)
    assert p.J == J
    print(f"adi_native n={n} J={J}", flush=True)
    Y = fps.adi_native(p, _dev(G)).cpu().numpy()
    Yo = square.adi_exact_iterate(G, po)
    parity.check(Y, Yo, 1e-10, f"adi_native n={n}")


@pytest.mark.parametrize("n", [1, 2, 3, 8, 64, 130, 513, 1024])
def test_solve_matches_exact_discrete_solution(n):
    F = workloads.square_rhs(n, seed=0)
    print(f"solve n={n}", flush=True)
    p = fps.plan(n, tol=1e-13)
    U = fps.solve(p, _dev(F))
    torch.cuda.synchronize()
    Uo = square.poisson_square(F)
    assert U.shape == (n + 2, n + 2)
    parity.check(U.cpu().numpy(), Uo, 1e-12, f"solve n={n}")


@pytest.mark.parametrize("n", [7, 64, 300])
def test_native_output_matches(n):
    F = workloads.square_rhs(n, seed=3)
    p = fps.plan(n, tol=1e-13, out="native")
    X = fps.solve(p, _dev(F))
    torch.cuda.synchronize()
    Xo = square.poisson_square(F, out="native")
    parity.check(X.cpu().numpy(), Xo, 1e-12, f"native n={n}")


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


@pytest.mark.parametrize("precision,out,box", [("fp64", "cheb", None),
                                               ("fp32_refined", "cheb", None),
                                               ("fp64", "native", None),
                                               ("fp32_refined", "native", None),
                                               ("fp64", "cheb", (0.0, 2.5, -1.0, 0.25))])
def test_row_parity_streams_equal_one_stream(precision, out, box):
    # Chains of more than two chunks (n > 256): a solve runs its two
    # row-parity blocks (the ADI, or the refinement rounds) on two streams;
    # with sweep timing on, every launch goes to the caller's stream instead.  The same kernels see the same data either way, so the
    # results agree bit for bit.
    for n in (300, 1030, 2100):
        print(f"streams n={n} {precision} {out} box={box}", flush=True)
        p = fps.plan(n, tol=1e-13, precision=precision, out=out, box=box)
        F = _dev(workloads.square_rhs(n, seed=3, decay=0.0))
        U2 = fps.solve(p, F).clone()
        p.set_sweep_timing(2)
        U1 = fps.solve(p, F)
        torch.cuda.synchronize()
        p.set_sweep_timing(0)
        assert torch.equal(U1, U2)
        if precision != "fp64" or out != "cheb" or box is not None:
            continue
        Y2 = fps.adi_native(p, F).clone()
        p.set_sweep_timing(2)
        Y1 = fps.adi_native(p, F)
        torch.cuda.synchronize()
        p.set_sweep_timing(0)
        assert torch.equal(Y1, Y2)


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
    parity.check(Ug, Uo, 1e-12, "n=4096")


@pytest.mark.parametrize("n", [1030, 4096])
def test_undecayed_input_full_parity(n):
    # F with N(0,1) entries of the same size at every index: the high-index
    # coefficients, where the maps' triangular skips, edge tiles and padding
    # act, weigh as much as the low ones.
    F = workloads.square_rhs(n, seed=7, decay=0.0)
    print(f"undecayed n={n}", flush=True)
    p = fps.plan(n, tol=1e-13, tight=True)
    U = fps.solve(p, _dev(F)).cpu().numpy()
    parity.check(U, square.poisson_square(F), 1e-12, f"undecayed n={n}")
    X = fps.solve(fps.plan(n, tol=1e-13, tight=True, out="native"), _dev(F)).cpu().numpy()
    parity.check(X, square.poisson_square(F, out="native"), 1e-12, f"undecayed native n={n}")


def test_largest_workload_size_full_parity():
    # n = 10^4 (10^8 dof): full comparison with the oracle (measured 6.6e-14).
    n = 10000
    F = workloads.square_rhs(n, seed=0)
    print("n=10000 solve", flush=True)
    p = fps.plan(n, tol=1e-13, tight=True)
    U = fps.solve(p, _dev(F)).cpu().numpy()
    print("n=10000 oracle", flush=True)
    Uo = square.poisson_square(F)
    parity.check(U, Uo, 1e-12, "n=10000")


@pytest.mark.parametrize("n", [1, 5, 64, 300, 1024, 4096])
def test_tight_spectrum_solve_matches_exact(n):
    # Shift intervals from the computed spectrum (fewer iterations, same bound).
    F = workloads.square_rhs(n, seed=0)
    p = fps.plan(n, tol=1e-13, tight=True)
    print(f"tight n={n} J={p.J}", flush=True)
    U = fps.solve(p, torch.from_numpy(F).cuda())
    torch.cuda.synchronize()
    Uo = square.poisson_square(F)
    parity.check(U.cpu().numpy(), Uo, 1e-12, f"tight n={n}")
