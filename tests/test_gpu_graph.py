"""A single-plan solve captured into a HIP graph: every replay (with eager
work on the device between replays) equals the eager solve bit for bit,
and a new input written into the captured buffer gives the new solution."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
import paper_1710_11259_amd as fps  # noqa: E402

pytestmark = pytest.mark.gpu


def _inputs(kind, n, seed):
    if kind == "cylinder":
        F = workloads.cylinder_rhs(n, 8, seed=seed)
        return np.ascontiguousarray(np.stack([F.real, F.imag], axis=1))
    if kind.startswith("cube"):
        return workloads.cube_rhs(n, seed=seed)
    return workloads.square_rhs(n, seed=seed)


def _plan(kind, n):
    if kind == "square":
        return fps.plan(n, tol=1e-13, tight=True)
    if kind == "square_refined":
        return fps.plan(n, tol=1e-13, precision="fp32_refined")
    if kind == "rect":
        return fps.plan(n, tol=1e-13, box=(0.0, 2.5, -1.0, 0.25))
    if kind == "cube_zeig":
        return fps.plan(n, tol=1e-13, dim=3, tight=True, zeig=True)
    if kind == "cube":
        return fps.plan(n, tol=1e-13, dim=3, tight=True)
    return fps.plan_cylinder(n, 8)


# cube_zeig at n = 200 runs its 58 longest slices on the plan's second
# stream, so the capture also records the fork and join between streams.
@pytest.mark.parametrize("kind,n", [("square", 64), ("square", 300), ("square", 1024),
                                    ("square_refined", 200), ("rect", 130),
                                    ("cube_zeig", 33), ("cube_zeig", 200), ("cube", 12),
                                    ("cylinder", 40)])
def test_solve_graph_replays_match_eager(kind, n):
    print(f"graph {kind} n={n}", flush=True)
    p = _plan(kind, n)
    F1 = torch.from_numpy(_inputs(kind, n, 1)).cuda()
    ref1 = fps.solve(p, F1).cpu().numpy()
    g = fps.SolveGraph(p)
    for rep in range(3):
        g.F.copy_(F1)
        out = g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref1), f"replay {rep}"
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum()
        torch.cuda.synchronize()
        del junk
    F2 = torch.from_numpy(_inputs(kind, n, 2)).cuda()
    ref2 = fps.solve(p, F2).cpu().numpy()
    g.F.copy_(F2)
    out = g.replay()
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref2)
    assert not np.array_equal(ref1, ref2)
