"""GPU parity of the batched square solve: every problem of a batch equals
the single-problem solve of the same size bit for bit (same kernels, same
per-problem arithmetic), and the exact discrete solution of the oracle."""
import numpy as np
import pytest

import parity
import workloads
from oracle import square

torch = pytest.importorskip("torch")
import paper_1710_11259_amd as fps  # noqa: E402

pytestmark = pytest.mark.gpu

MIXED = [1, 5, 64, 129, 32, 544, 64, 300, 2, 1030]


def _rhs(ns, seed=7):
    rng = np.random.default_rng(seed)
    return [workloads.decayed_normal(rng, (n, n), 1.5) for n in ns]


def _single(n, F, **kw):
    p = fps.plan(n, **kw)
    U = fps.solve(p, torch.from_numpy(F).cuda())
    torch.cuda.synchronize()
    return U.cpu().numpy()


@pytest.mark.parametrize("out,precision", [("cheb", "fp64"), ("native", "fp64"),
                                           ("cheb", "fp32_refined"), ("native", "fp32_refined")])
def test_batch_equals_single_solves_bitwise(out, precision):
    Fs = _rhs(MIXED)
    b = fps.batch(MIXED, tol=1e-13, out=out, precision=precision)
    print(f"batch {precision} {out}: {len(MIXED)} problems, max J {b.max_J}", flush=True)
    U = fps.batch_solve(b, b.pack(Fs))
    torch.cuda.synchronize()
    Us = [u.cpu().numpy() for u in b.unpack(U)]
    for n, F, Ub in zip(MIXED, Fs, Us):
        Ur = _single(n, F, tol=1e-13, out=out, precision=precision)
        assert Ub.shape == Ur.shape
        assert np.array_equal(Ub, Ur), f"n={n}: batched result differs from the single solve"
    for n, F, Ub in zip(MIXED, Fs, Us):
        if n <= 300:
            Uo = square.poisson_square(F, out=out)
            parity.check(Ub, Uo, 1e-12, f"n={n}")


@pytest.mark.parametrize("out", ["cheb", "native"])
def test_batch_adjoint_equals_single_adjoints_bitwise(out):
    # the batched adjoint (fps_batch_solve_adjoint): per-problem transposed
    # maps around the batched ADI, so each problem equals fps_solve_adjoint
    rng = np.random.default_rng(11)
    Ubs = [rng.standard_normal((n + 2, n + 2) if out == "cheb" else (n, n)) for n in MIXED]
    b = fps.batch(MIXED, tol=1e-13, out=out)
    print(f"batch adjoint {out}: {len(MIXED)} problems", flush=True)
    Ub_packed = torch.cat([torch.from_numpy(u).reshape(-1) for u in Ubs]).cuda()
    Fb = fps.batch_solve_adjoint(b, Ub_packed)
    torch.cuda.synchronize()
    Fb = Fb.cpu().numpy()
    for i, (n, Ub) in enumerate(zip(MIXED, Ubs)):
        p = fps.plan(n, tol=1e-13, out=out)
        ref = fps.solve_adjoint(p, torch.from_numpy(Ub).cuda()).cpu().numpy()
        got = Fb[b.in_offsets[i]:b.in_offsets[i + 1]].reshape(n, n)
        assert np.array_equal(got, ref), f"n={n}: batched adjoint differs from the single adjoint"


def test_batch_adjoint_rejects_refined_batch():
    b = fps.batch([8, 16], tol=1e-13, precision="fp32_refined")
    Ub = torch.zeros(b.out_entries, dtype=torch.float64, device="cuda")
    with pytest.raises(fps.FpsError) as e:
        fps.batch_solve_adjoint(b, Ub)
    assert e.value.status == fps.FPS_E_UNSUPPORTED


def test_batch_refined_matches_oracle():
    ns = [1, 5, 64, 129, 544, 1024, 32]
    Fs = _rhs(ns, seed=8)
    b = fps.batch(ns, tol=1e-13, precision="fp32_refined")
    print(f"batch refined: max J {b.max_J}", flush=True)
    U = fps.batch_solve(b, b.pack(Fs))
    torch.cuda.synchronize()
    for n, F, Ub in zip(ns, Fs, b.unpack(U)):
        Uo = square.poisson_square(F)
        Ub = Ub.cpu().numpy()
        parity.check(Ub, Uo, 1e-12, f"refined n={n}")


def test_batch_workload_256_problems():
    # 256 problems, n_b = 32 U{1..32}, seed 1 (the batched workload).
    ns, Fs = workloads.batched_problems()
    b = fps.batch(ns, tol=1e-13)
    print(f"256-problem batch: sum n^2 = {sum(n * n for n in ns)}, max J {b.max_J}", flush=True)
    U = fps.batch_solve(b, b.pack(Fs))
    torch.cuda.synchronize()
    Us = b.unpack(U)
    # bitwise against single solves for one problem of every distinct size
    seen = set()
    for i, n in enumerate(ns):
        if n in seen:
            continue
        seen.add(n)
        Ur = _single(n, Fs[i], tol=1e-13)
        assert np.array_equal(Us[i].cpu().numpy(), Ur), f"problem {i} (n={n})"
    # against the oracle on a sample spanning the sizes
    order = np.argsort(ns)
    for i in order[:: max(1, len(ns) // 8)]:
        Uo = square.poisson_square(Fs[i])
        parity.check(Us[i].cpu().numpy(), Uo, 1e-12)


def test_batch_workload_256_problems_refined():
    # The FP32-refined batch of the 256-problem workload: bit-identical to the
    # refined single solves for one problem of every size, and against the
    # oracle on a sample spanning the sizes.
    ns, Fs = workloads.batched_problems()
    b = fps.batch(ns, tol=1e-13, precision="fp32_refined")
    print(f"256-problem refined batch, max J {b.max_J}", flush=True)
    U = fps.batch_solve(b, b.pack(Fs))
    torch.cuda.synchronize()
    Us = b.unpack(U)
    seen = set()
    for i, n in enumerate(ns):
        if n in seen or len(seen) >= 8:
            continue
        seen.add(n)
        Ur = _single(n, Fs[i], tol=1e-13, precision="fp32_refined")
        assert np.array_equal(Us[i].cpu().numpy(), Ur), f"problem {i} (n={n})"
    order = np.argsort(ns)
    for i in order[:: max(1, len(ns) // 10)]:
        parity.check(Us[i].cpu().numpy(), square.poisson_square(Fs[i]), 1e-12,
                     f"refined problem {i} n={ns[i]}")


def test_batch_graph_replays_match_eager():
    ns = [32, 96, 64, 160, 512, 33]
    Fs = _rhs(ns, seed=9)
    b = fps.batch(ns, tol=1e-13)
    g = fps.BatchGraph(b)
    ref = fps.batch_solve(b, b.pack(Fs)).cpu().numpy()
    for rep in range(3):
        g.F.copy_(b.pack(Fs))
        out = g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), f"replay {rep}"
        # eager work on the same stream between replays
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum()
        torch.cuda.synchronize()
        del junk
    # a different input through the same graph
    Fs2 = _rhs(ns, seed=10)
    g.F.copy_(b.pack(Fs2))
    out = g.replay()
    torch.cuda.synchronize()
    ref2 = fps.batch_solve(b, b.pack(Fs2)).cpu().numpy()
    assert np.array_equal(out.cpu().numpy(), ref2)
