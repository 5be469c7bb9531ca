"""GPU parity of the FP32-storage / FP64-refinement form against the oracle."""
import numpy as np
import pytest

import workloads
from oracle import square

torch = pytest.importorskip("torch")
import paper_1710_11259_amd as fps  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.mark.parametrize("n,out", [(1, "cheb"), (5, "cheb"), (64, "cheb"), (129, "cheb"),
                                   (300, "native"), (1024, "cheb")])
def test_refined_matches_exact_discrete_solution(n, out):
    F = workloads.square_rhs(n, seed=0)
    p = fps.plan(n, tol=1e-13, precision="fp32_refined", out=out)
    print(f"refined n={n} J_inner={p.J}", flush=True)
    U = fps.solve(p, _dev(F))
    torch.cuda.synchronize()
    Uo = square.poisson_square(F, out="native" if out == "native" else "cheb")
    err = np.linalg.norm(U.cpu().numpy() - Uo) / np.linalg.norm(Uo)
    print(f"rel err {err:.3e}", flush=True)
    assert err <= 1e-12


def test_refined_headline_size():
    n = 4096
    F = workloads.square_rhs(n, seed=0)
    p = fps.plan(n, tol=1e-13, precision="fp32_refined")
    U = fps.solve(p, _dev(F))
    torch.cuda.synchronize()
    Uo = square.poisson_square(F)
    err = np.linalg.norm(U.cpu().numpy() - Uo) / np.linalg.norm(Uo)
    print(f"refined n=4096 rel err {err:.3e}", flush=True)
    assert err <= 1e-12
