"""Every solve must read only workspace it wrote during the same call: run
each form on a workspace pre-filled with NaN bytes and compare with the
oracle (any stale read propagates a NaN)."""
import numpy as np
import pytest

import parity
import workloads
from oracle import cube, square

torch = pytest.importorskip("torch")
import paper_1710_11259_amd as fps  # noqa: E402

pytestmark = pytest.mark.gpu


def _nan_ws(p):
    return torch.full((max(p.workspace_bytes, 256),), 0xFF, dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("n,out", [(1, "cheb"), (2, "native"), (5, "cheb"), (64, "cheb")])
@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_square_ignores_stale_workspace(n, out, precision):
    F = workloads.square_rhs(n, seed=0)
    p = fps.plan(n, tol=1e-13, out=out, precision=precision)
    U = fps.solve(p, torch.from_numpy(F).cuda(), ws=_nan_ws(p))
    torch.cuda.synchronize()
    Uo = square.poisson_square(F, out=out)
    parity.check(U.cpu().numpy(), Uo, 1e-12)


@pytest.mark.parametrize("n,out", [(1, "cheb"), (2, "cheb"), (5, "native"), (17, "cheb")])
@pytest.mark.parametrize("zeig", [False, True])
def test_cube_ignores_stale_workspace(n, out, zeig):
    F = workloads.cube_rhs(n)
    p = fps.plan(n, tol=1e-13, dim=3, out=out, zeig=zeig)
    U = fps.solve(p, torch.from_numpy(F).cuda(), ws=_nan_ws(p))
    torch.cuda.synchronize()
    Uo = cube.poisson_cube(F, out=out)
    parity.check(U.cpu().numpy(), Uo, 1e-12)


def test_batch_ignores_stale_workspace():
    ns = [1, 2, 5, 64, 33]
    rng = np.random.default_rng(11)
    Fs = [workloads.decayed_normal(rng, (n, n), 1.5) for n in ns]
    b = fps.batch(ns, tol=1e-13)
    ws = torch.full((b.workspace_bytes,), 0xFF, dtype=torch.uint8, device="cuda")
    U = fps.batch_solve(b, b.pack(Fs), ws=ws)
    torch.cuda.synchronize()
    for n, F, Ub in zip(ns, Fs, b.unpack(U)):
        Uo = square.poisson_square(F)
        parity.check(Ub.cpu().numpy(), Uo, 1e-12, f"n={n}")


def test_adjoint_ignores_stale_workspace():
    from oracle import adjoint
    n = 5
    p = fps.plan(n, tol=1e-13)
    Ub = np.random.default_rng(12).standard_normal(p.out_shape())
    Fb = fps.solve_adjoint(p, torch.from_numpy(Ub).cuda(), ws=_nan_ws(p))
    torch.cuda.synchronize()
    Fo = adjoint.vjp_square(Ub)
    parity.check(Fb.cpu().numpy(), Fo, 1e-12, "adjoint")


@pytest.mark.parametrize("n", [1, 2, 5, 64])
@pytest.mark.parametrize("box", [None, (0.0, 2.5, -1.0, 0.25)])
@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_dirichlet_ignores_stale_workspace(n, box, precision):
    from oracle import rect
    F, bc = workloads.rect_dirichlet_case(n, seed=5)
    p = fps.plan(n, tol=1e-13, box=box, precision=precision, dirichlet=True)
    U = fps.solve_dirichlet(p, torch.from_numpy(F).cuda(), torch.from_numpy(bc).cuda(),
                            ws=_nan_ws(p))
    torch.cuda.synchronize()
    Uo = rect.poisson_rect_dirichlet(F, bc, box or (-1.0, 1.0, -1.0, 1.0))
    parity.check(U.cpu().numpy(), Uo, 1e-12)
