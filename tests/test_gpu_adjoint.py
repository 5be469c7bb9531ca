"""GPU parity of the differentiable solve (adjoint / VJP) against the oracle."""
import numpy as np
import pytest

import parity
import workloads
from oracle import adjoint, basis, shifts as oshifts, square

torch = pytest.importorskip("torch")
import paper_1710_11259_amd as fps  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.mark.parametrize("n,out", [(1, "cheb"), (5, "cheb"), (64, "cheb"), (130, "cheb"),
                                   (257, "native"), (700, "cheb")])
def test_adjoint_matches_oracle_vjp(n, out):
    rng = np.random.default_rng(n)
    p = fps.plan(n, tol=1e-13, out=out)
    Ub = rng.standard_normal(p.out_shape())
    print(f"adjoint n={n} out={out}", flush=True)
    Fb = fps.solve_adjoint(p, _dev(Ub))
    torch.cuda.synchronize()
    _, po, _ = oshifts.square_shifts(n, 1e-13)
    if out == "cheb":
        ref = adjoint.vjp_square(Ub, po)
    else:
        # native map X = S^-1 Y_J(S^-1 R F R^T S^-1) S^-1, transposed
        s = square.s_diag(n)
        R = basis.cheb_to_ct(n)
        Gb = square.adi_exact_iterate(Ub / np.outer(s, s), po) / np.outer(s, s)
        ref = R.T @ Gb @ R
    parity.check(Fb.cpu().numpy(), ref, 1e-12)


@pytest.mark.parametrize("n", [33, 512])
def test_dot_product_identity_on_gpu(n):
    rng = np.random.default_rng(7)
    p = fps.plan(n, tol=1e-13)
    F = _dev(rng.standard_normal((n, n)))
    Ub = _dev(rng.standard_normal(p.out_shape()))
    U = fps.solve(p, F)
    Fb = fps.solve_adjoint(p, Ub)
    torch.cuda.synchronize()
    lhs = float((U * Ub).sum())
    rhs = float((F * Fb).sum())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_autograd_central_differences_batch():
    # loss = ||U(F) - U*||^2 over a batch; central differences with h = 1e-6 on
    # random unit directions (exact up to rounding for a quadratic loss).
    n, batch, ndirs = 256, 4, 8
    F, Fstar, dirs = workloads.adjoint_case(n, batch, n_dirs=ndirs)
    p = fps.plan(n, tol=1e-13)
    Ustar = fps.solve(p, _dev(Fstar))
    Ft = _dev(F).requires_grad_(True)
    U = fps.solve_fn(Ft, p)
    loss = ((U - Ustar) ** 2).sum()
    loss.backward()
    g = Ft.grad.detach()
    h = 1e-6

    def L(FF):
        with torch.no_grad():
            return float(((fps.solve_fn(FF, p) - Ustar) ** 2).sum())

    for d in range(ndirs):
        D = _dev(dirs[d])
        fd = (L(Ft.detach() + h * D) - L(Ft.detach() - h * D)) / (2 * h)
        an = float((g * D).sum())
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (d, fd, an)


def test_autograd_full_size_workload():
    # n = 2048, batch 16, loss ||U(F) - U*||^2, 32 unit directions, h = 1e-6.
    n, batch, ndirs = 2048, 16, 32
    F, Fstar, dirs = workloads.adjoint_case(n, batch, n_dirs=ndirs)
    p = fps.plan(n, tol=1e-13)
    print(f"autograd n={n} batch={batch} J={p.J}", flush=True)
    Ustar = fps.solve(p, _dev(Fstar))
    Ft = _dev(F).requires_grad_(True)
    loss = ((fps.solve_fn(Ft, p) - Ustar) ** 2).sum()
    loss.backward()
    g = Ft.grad.detach()
    h = 1e-6

    def L(FF):
        with torch.no_grad():
            return float(((fps.solve_fn(FF, p) - Ustar) ** 2).sum())

    worst = 0.0
    for d in range(ndirs):
        D = _dev(dirs[d])
        fd = (L(Ft.detach() + h * D) - L(Ft.detach() - h * D)) / (2 * h)
        an = float((g * D).sum())
        worst = max(worst, abs(fd - an) / max(1.0, abs(an)))
    print(f"worst relative FD mismatch {worst:.2e}", flush=True)
    assert worst <= 1e-6
