"""GPU parity of the FP32-storage / FP64-refinement form against the oracle:
relative Frobenius and max-abs / max-abs error of U (or X) <= 1e-12 against
the exact discrete solution, for the decayed workload input and for
undecayed N(0,1) input (every coefficient of F of the same size)."""
import numpy as np
import pytest

import workloads
from oracle import square

torch = pytest.importorskip("torch")
import paper_1710_11259_amd as fps  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _errs(U, Uo):
    return (np.linalg.norm(U - Uo) / np.linalg.norm(Uo), np.abs(U - Uo).max() / np.abs(Uo).max())


@pytest.mark.parametrize("n,out,decay", [(1, "cheb", 2.0), (5, "cheb", 2.0), (64, "cheb", 2.0),
                                         (129, "cheb", 2.0), (300, "native", 2.0),
                                         (1024, "cheb", 2.0), (1030, "cheb", 0.0),
                                         (2048, "native", 2.0), (2048, "cheb", 0.0)])
def test_refined_matches_exact_discrete_solution(n, out, decay):
    F = workloads.square_rhs(n, seed=0, decay=decay)
    p = fps.plan(n, tol=1e-13, precision="fp32_refined", out=out)
    print(f"refined n={n} decay={decay} rounds {p.round_steps()}", flush=True)
    U = fps.solve(p, _dev(F))
    torch.cuda.synchronize()
    Uo = square.poisson_square(F, out="native" if out == "native" else "cheb")
    err, emax = _errs(U.cpu().numpy(), Uo)
    print(f"rel err {err:.3e} max-abs {emax:.3e}", flush=True)
    assert err <= 1e-12 and emax <= 1e-12


@pytest.mark.parametrize("tight", [False, True])
def test_refined_headline_size(tight):
    n = 4096
    F = workloads.square_rhs(n, seed=0)
    p = fps.plan(n, tol=1e-13, precision="fp32_refined", tight=tight)
    print(f"refined n=4096 tight={tight} rounds {p.round_steps()}", flush=True)
    U = fps.solve(p, _dev(F))
    torch.cuda.synchronize()
    Uo = square.poisson_square(F)
    err, emax = _errs(U.cpu().numpy(), Uo)
    print(f"refined n=4096 rel err {err:.3e} max-abs {emax:.3e}", flush=True)
    assert err <= 1e-12 and emax <= 1e-12


@pytest.mark.parametrize("tol,bar", [(1e-10, 1e-9), (1e-6, 1e-5)])
def test_refined_looser_targets(tol, bar):
    # fewer rounds for a looser tolerance, error still within it
    n = 700
    F = workloads.square_rhs(n, seed=3)
    p = fps.plan(n, tol=tol, precision="fp32_refined")
    assert p.rounds == 2
    U = fps.solve(p, _dev(F))
    torch.cuda.synchronize()
    err, emax = _errs(U.cpu().numpy(), square.poisson_square(F))
    print(f"refined tol={tol} rel err {err:.3e} max-abs {emax:.3e}", flush=True)
    assert err <= bar and emax <= bar
