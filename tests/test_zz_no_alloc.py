"""The allocation-free solve (fps_solve_noalloc, workspace in the library's
static device scratch) against fps_solve on a caller-owned workspace and the
oracle: two calls in a row, the second smaller, so the second runs on the
scratch contents the first left behind."""
import ctypes

import numpy as np
import pytest

import workloads
from oracle import rect, square

torch = pytest.importorskip("torch")
import paper_1710_11259_amd as fps  # noqa: E402

pytestmark = pytest.mark.gpu

BOX = (0.0, 2.5, -1.0, 0.25)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b), np.abs(a - b).max() / np.abs(b).max()


def _pair(p, F):
    Fd = torch.from_numpy(F).cuda()
    U_ref = fps.solve(p, Fd)
    U_na = fps.solve_noalloc(p, Fd)
    torch.cuda.synchronize()
    return U_na.cpu().numpy(), U_ref.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_noalloc_square_two_calls_second_smaller(precision):
    for n in (1030, 300):
        print(f"noalloc square n={n} {precision}", flush=True)
        F = workloads.square_rhs(n, seed=0)
        p = fps.plan(n, tol=1e-13, precision=precision)
        assert p.workspace_bytes <= fps.noalloc_capacity()
        U_na, U_ref = _pair(p, F)
        # same kernels on the same inputs: bit for bit
        assert np.array_equal(U_na, U_ref)
        fro, mx = _rel(U_na, square.poisson_square(F))
        assert fro <= 1e-12 and mx <= 1e-12


def test_noalloc_rect_native_then_smaller_square():
    n = 700
    print(f"noalloc rect n={n}", flush=True)
    F = workloads.square_rhs(n, seed=5)
    p = fps.Plan(n, tol=1e-13, box=BOX, out="native")
    U_na, U_ref = _pair(p, F)
    assert np.array_equal(U_na, U_ref)
    fro, mx = _rel(U_na, rect.poisson_rect(F, BOX, out="native"))
    assert fro <= 1e-12 and mx <= 1e-12
    n = 65
    print(f"noalloc square n={n}", flush=True)
    F = workloads.square_rhs(n, seed=1)
    p = fps.plan(n, tol=1e-13)
    U_na, U_ref = _pair(p, F)
    assert np.array_equal(U_na, U_ref)


def test_noalloc_rejects_plans_beyond_the_scratch():
    L = fps.lib()
    F = torch.zeros(1, dtype=torch.float64, device="cuda")
    U = torch.zeros(1, dtype=torch.float64, device="cuda")
    big = fps.plan(2048, tol=1e-13)
    assert big.workspace_bytes > fps.noalloc_capacity()
    st = L.fps_solve_noalloc(big.handle, ctypes.c_void_p(F.data_ptr()),
                             ctypes.c_void_p(U.data_ptr()), None)
    assert st == fps.FPS_E_UNSUPPORTED
    assert b"exceeds" in L.fps_last_error()
    cube = fps.plan(5, tol=1e-13, dim=3)
    st = L.fps_solve_noalloc(cube.handle, ctypes.c_void_p(F.data_ptr()),
                             ctypes.c_void_p(U.data_ptr()), None)
    assert st == fps.FPS_E_UNSUPPORTED
