"""GPU parity of the rectangle solver (general-interval shifts, two tables
per ADI step) and of nonhomogeneous Dirichlet data against the oracle."""
import numpy as np
import pytest

import parity
import workloads
from oracle import basis, rect, square

torch = pytest.importorskip("torch")
import paper_1710_11259_amd as fps  # noqa: E402

pytestmark = pytest.mark.gpu

BOXES = [(0.0, 2.5, -1.0, 0.25), (0.0, 10.0, 0.0, 1.0)]
UNIT = (-1.0, 1.0, -1.0, 1.0)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.mark.parametrize("box", BOXES)
@pytest.mark.parametrize("n,tol", [(1, 1e-13), (2, 1e-13), (5, 1e-13), (16, 1e-6), (64, 1e-13),
                                   (257, 1e-10), (600, 1e-13)])
def test_rect_adi_iterate_matches_closed_form(n, tol, box):
    # Algorithm 2's J-step iterate for A = sx2 A~, B = -sy2 A~ in closed form
    # (any shifts): pins the two-table sweeps and the general pass
    # coefficients independently of convergence.
    rng = np.random.default_rng(n)
    G = rng.standard_normal((n, n)) / np.outer(np.arange(1, n + 1), np.arange(1, n + 1))
    p = fps.plan(n, tol=tol, box=box)
    J, po, qo = rect.rect_shifts(n, box, tol)
    assert p.J == J
    print(f"rect adi_native n={n} tol={tol} box={box} J={J}", flush=True)
    Y = fps.adi_native(p, _dev(G))
    torch.cuda.synchronize()
    Yo = rect.adi_iterate_rect(G, box, po, qo)
    parity.check(Y.cpu().numpy(), Yo, 1e-12, f"rect adi_native n={n}")


@pytest.mark.parametrize("box", BOXES)
@pytest.mark.parametrize("n", [1, 2, 3, 8, 64, 130, 513, 1024])
def test_rect_solve_matches_exact_discrete_solution(n, box):
    F = workloads.square_rhs(n, seed=0)
    print(f"rect solve n={n} box={box}", flush=True)
    U = fps.solve(fps.plan(n, tol=1e-13, box=box), _dev(F))
    torch.cuda.synchronize()
    parity.check(U.cpu().numpy(), rect.poisson_rect(F, box), 1e-12)


@pytest.mark.parametrize("box", BOXES)
def test_rect_native_tight_and_refined(box):
    n = 300
    F = workloads.square_rhs(n, seed=2)
    Xo = rect.poisson_rect(F, box, out="native")
    Uo = rect.poisson_rect(F, box)
    for kw, ref in (({"out": "native"}, Xo), ({"tight": True}, Uo),
                    ({"precision": "fp32_refined"}, Uo),
                    ({"precision": "fp32_refined", "tight": True}, Uo)):
        print(f"rect n={n} box={box} {kw}", flush=True)
        U = fps.solve(fps.plan(n, tol=1e-13, box=box, **kw), _dev(F))
        torch.cuda.synchronize()
        parity.check(U.cpu().numpy(), ref, 1e-12)


def test_rect_full_size():
    n = 4096
    box = BOXES[0]
    F = workloads.square_rhs(n, seed=0)
    print("rect n=4096 fp64 tight", flush=True)
    U = fps.solve(fps.plan(n, tol=1e-13, box=box, tight=True), _dev(F))
    torch.cuda.synchronize()
    parity.check(U.cpu().numpy(), rect.poisson_rect(F, box), 1e-12)


@pytest.mark.parametrize("box", [None] + BOXES)
@pytest.mark.parametrize("n", [1, 2, 7, 64, 257, 1024])
def test_dirichlet_matches_oracle(n, box):
    F, bc = workloads.rect_dirichlet_case(n, seed=5)
    print(f"dirichlet n={n} box={box}", flush=True)
    p = fps.plan(n, tol=1e-13, box=box, dirichlet=True)
    U = fps.solve_dirichlet(p, _dev(F), _dev(bc))
    torch.cuda.synchronize()
    Uo = rect.poisson_rect_dirichlet(F, bc, box or UNIT)
    Ug = U.cpu().numpy()
    parity.check(Ug, Uo, 1e-12, f"dirichlet n={n}")
    for got, want in zip(rect.boundary_traces(Ug), bc):
        assert np.abs(got - want).max() <= 1e-12 * np.abs(bc).max()


@pytest.mark.parametrize("n", [200, 1024])
@pytest.mark.parametrize("box", [None, BOXES[1]])
def test_dirichlet_refined_and_tight(box, n):
    F, bc = workloads.rect_dirichlet_case(n, seed=9)
    Uo = rect.poisson_rect_dirichlet(F, bc, box or UNIT)
    for kw in ({"precision": "fp32_refined"}, {"tight": True}):
        print(f"dirichlet n={n} box={box} {kw}", flush=True)
        U = fps.solve_dirichlet(fps.plan(n, tol=1e-13, box=box, dirichlet=True, **kw), _dev(F),
                                _dev(bc))
        torch.cuda.synchronize()
        parity.check(U.cpu().numpy(), Uo, 1e-12, f"dirichlet n={n} {kw}")


def test_dirichlet_full_size():
    # n = 4096, the benchmark's rectangle and random traces (coefficients ~ k^-2)
    n = 4096
    box = BOXES[0]
    F, bc = workloads.rect_dirichlet_case(n, seed=5)
    print("dirichlet n=4096 tight", flush=True)
    U = fps.solve_dirichlet(fps.plan(n, tol=1e-13, box=box, tight=True, dirichlet=True), _dev(F),
                            _dev(bc))
    torch.cuda.synchronize()
    Ug = U.cpu().numpy()
    for got, want in zip(rect.boundary_traces(Ug), bc):
        assert np.abs(got - want).max() <= 1e-12 * np.abs(bc).max()
    Uo = rect.poisson_rect_dirichlet(F, bc, box)
    parity.check(Ug, Uo, 1e-12, "dirichlet n=4096")


def test_dirichlet_manufactured_solution():
    box = BOXES[0]
    n = 40
    F, bc, u_fun = workloads.manufactured_rect(n, box)
    U = fps.solve_dirichlet(fps.plan(n, tol=1e-14, box=box, dirichlet=True), _dev(F), _dev(bc))
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    s, t = rng.uniform(-1, 1, 200), rng.uniform(-1, 1, 200)
    assert np.abs(basis.cheb_eval_2d(U.cpu().numpy(), s, t) - u_fun(s, t)).max() < 1e-11


def test_dirichlet_zero_data_equals_solve():
    n = 130
    box = BOXES[1]
    F = _dev(workloads.square_rhs(n, seed=4))
    p = fps.plan(n, tol=1e-13, box=box, dirichlet=True)
    U0 = fps.solve(p, F)
    U1 = fps.solve_dirichlet(p, F, torch.zeros((4, n + 2), dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert torch.equal(U0, U1)


def test_dirichlet_rejects_native_and_cube_plans():
    n = 8
    F = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    bc = torch.zeros((4, n + 2), dtype=torch.float64, device="cuda")
    with pytest.raises(fps.FpsError):
        fps.solve_dirichlet(fps.plan(n, out="native", dirichlet=True), F, bc,
                            out=torch.empty((n, n), dtype=torch.float64, device="cuda"))
    with pytest.raises(fps.FpsError):  # plan without the lift map
        fps.solve_dirichlet(fps.plan(n), F, bc)
    c = fps.plan(n, dim=3)
    with pytest.raises(fps.FpsError):
        import ctypes
        ws = fps.workspace(c)
        U = torch.empty((n + 2,) * 3, dtype=torch.float64, device="cuda")
        fps._check(fps.lib().fps_solve_dirichlet(c.handle, ctypes.c_void_p(F.data_ptr()),
                                                 ctypes.c_void_p(bc.data_ptr()),
                                                 ctypes.c_void_p(U.data_ptr()),
                                                 ctypes.c_void_p(ws.data_ptr()), None))


@pytest.mark.parametrize("n", [5, 64, 257])
def test_rect_adjoint_matches_oracle_vjp(n):
    box = BOXES[0]
    rng = np.random.default_rng(n)
    p = fps.plan(n, tol=1e-13, box=box)
    Ub = rng.standard_normal(p.out_shape())
    Fb = fps.solve_adjoint(p, _dev(Ub))
    torch.cuda.synchronize()
    # transpose of F -> P S^-1 Y_J(S^-1 R F R^T S^-1) S^-1 P^T, with the J-step
    # map self-adjoint (a multiplier in the eigenbasis of A~)
    _, po, qo = rect.rect_shifts(n, box, 1e-13)
    s = square.s_diag(n)
    P = basis.recombined_to_cheb(n)
    R = basis.cheb_to_ct(n)
    Gb = rect.adi_iterate_rect((P.T @ Ub @ P) / np.outer(s, s), box, po, qo) / np.outer(s, s)
    ref = R.T @ Gb @ R
    parity.check(Fb.cpu().numpy(), ref, 1e-12)


def test_rect_dot_product_identity():
    n = 300
    rng = np.random.default_rng(3)
    p = fps.plan(n, tol=1e-13, box=BOXES[1])
    F = _dev(rng.standard_normal((n, n)))
    Ub = _dev(rng.standard_normal(p.out_shape()))
    U = fps.solve(p, F)
    Fb = fps.solve_adjoint(p, Ub)
    torch.cuda.synchronize()
    lhs, rhs = float((U * Ub).sum()), float((F * Fb).sum())
    print(f"lhs {lhs:.16e} rhs {rhs:.16e}", flush=True)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
