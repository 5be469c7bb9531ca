"""GPU parity of the cube solve (two-level nested ADI, FP64) against the
oracle's exact eigen-decomposition solution of the cube system (5.2)."""
import numpy as np
import pytest

import parity
import workloads
from oracle import cube

torch = pytest.importorskip("torch")
import paper_1710_11259_amd as fps  # noqa: E402

pytestmark = pytest.mark.gpu


def _solve(n, F, out="cheb", tol=1e-13):
    p = fps.plan(n, tol=tol, dim=3, out=out)
    print(f"cube n={n} out={out} J_outer={p.J} ws={p.workspace_bytes / 2**20:.1f} MiB",
          flush=True)
    U = fps.solve(p, torch.from_numpy(np.ascontiguousarray(F)).cuda())
    torch.cuda.synchronize()
    return U.cpu().numpy()


@pytest.mark.parametrize("n,out", [(1, "cheb"), (2, "cheb"), (5, "native"), (16, "cheb"),
                                   (33, "cheb"), (64, "native"), (100, "cheb")])
def test_cube_matches_exact_discrete_solution(n, out):
    F = workloads.cube_rhs(n)
    U = _solve(n, F, out)
    Uo = cube.poisson_cube(F, out=out)
    parity.check(U, Uo, 1e-12)


def test_cube_manufactured_solution():
    # u = (1-x^2)(1-y^2)(1-z^2) cos(x y z^2), the paper's cube example.
    n = 24
    F, u_fun = workloads.manufactured_cube(n, N=40)
    U = _solve(n, F)
    Uex = workloads.cheb_coeffs_3d(u_fun, n + 2)
    err = np.abs(U - Uex).max()
    print(f"manufactured max coefficient err {err:.3e}", flush=True)
    assert err <= 1e-12


def test_cube_headline_size():
    n = 256
    F = workloads.cube_rhs(n)
    U = _solve(n, F)
    Uo = cube.poisson_cube(F)
    parity.check(U, Uo, 1e-12)


@pytest.mark.parametrize("n", [5, 64, 256])
def test_cube_tight_spectrum_matches_exact(n):
    F = workloads.cube_rhs(n)
    p = fps.plan(n, tol=1e-13, dim=3, tight=True)
    print(f"cube tight n={n} J_outer={p.J} inner={sum(p.inner_counts())}", flush=True)
    U = fps.solve(p, torch.from_numpy(F).cuda())
    torch.cuda.synchronize()
    Uo = cube.poisson_cube(F)
    parity.check(U.cpu().numpy(), Uo, 1e-12)


@pytest.mark.parametrize("n,out,tight", [(1, "cheb", False), (2, "cheb", True), (5, "native", True),
                                         (16, "cheb", False), (33, "cheb", True),
                                         (64, "native", True), (100, "cheb", True),
                                         (256, "cheb", True), (256, "cheb", False)])
def test_cube_zeig_matches_exact(n, out, tight):
    # z-eigenbasis method: per-slice ADI after an eigen-transform along z.
    F = workloads.cube_rhs(n)
    p = fps.plan(n, tol=1e-13, dim=3, out=out, tight=tight, zeig=True)
    print(f"cube zeig n={n} out={out} tight={tight} J_max={p.J} "
          f"slice steps={sum(p.slice_counts())}", flush=True)
    U = fps.solve(p, torch.from_numpy(F).cuda())
    torch.cuda.synchronize()
    Uo = cube.poisson_cube(F, out=out)
    parity.check(U.cpu().numpy(), Uo, 1e-12)


def test_cube_zeig_manufactured_solution():
    n = 24
    F, u_fun = workloads.manufactured_cube(n, N=40)
    U = _solve_zeig(n, F)
    Uex = workloads.cheb_coeffs_3d(u_fun, n + 2)
    assert np.abs(U - Uex).max() <= 1e-12


def _solve_zeig(n, F):
    p = fps.plan(n, tol=1e-13, dim=3, tight=True, zeig=True)
    U = fps.solve(p, torch.from_numpy(np.ascontiguousarray(F)).cuda())
    torch.cuda.synchronize()
    return U.cpu().numpy()


@pytest.mark.parametrize("n", [9, 64, 256])
def test_cube_zeig_two_streams_equal_one(n):
    # The plan runs its longest slices on a second stream; with per-launch
    # timing on, every launch goes to the caller's stream.  Each slice's
    # arithmetic is the same either way, so the results agree bit for bit.
    F = torch.from_numpy(workloads.cube_rhs(n)).cuda()
    p = fps.plan(n, tol=1e-13, dim=3, tight=True, zeig=True)
    print(f"cube zeig streams n={n}", flush=True)
    U2 = fps.solve(p, F)
    p.set_sweep_timing(4 * max(p.slice_counts()))
    U1 = fps.solve(p, F)
    torch.cuda.synchronize()
    p.sweep_time()
    p.set_sweep_timing(0)
    U3 = fps.solve(p, F)
    torch.cuda.synchronize()
    assert torch.equal(U1, U2)
    assert torch.equal(U3, U2)


_ORACLE = {}


def _oracle(n):
    if n not in _ORACLE:
        print(f"oracle n={n}", flush=True)
        _ORACLE[n] = cube.poisson_cube(workloads.cube_rhs(n))
    return _ORACLE[n]


@pytest.mark.parametrize("n,zeig,precision", [(384, False, "fp64"), (384, True, "fp64"),
                                              (384, True, "fp32_refined"), (512, True, "fp64"),
                                              (512, True, "fp32_refined")])
def test_cube_largest_sizes_match_exact(n, zeig, precision):
    # the largest sizes each cube method accepts (nested 384, z-eigenbasis
    # 512, whose two-stream split puts the most slices on the second stream)
    F = torch.from_numpy(workloads.cube_rhs(n)).cuda()
    p = fps.plan(n, tol=1e-13, dim=3, tight=True, zeig=zeig, precision=precision)
    print(f"cube n={n} zeig={zeig} {precision} ws={p.workspace_bytes / 2**30:.2f} GiB", flush=True)
    U = fps.solve(p, F).cpu().numpy()
    del p, F
    torch.cuda.empty_cache()
    parity.check(U, _oracle(n), 1e-12, f"cube n={n} zeig={zeig} {precision}")

