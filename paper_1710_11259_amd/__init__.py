"""MI355X (gfx950) spectral fast Poisson solver.

Fortunato & Townsend, "Fast Poisson solvers for spectral methods"
(arXiv 1710.11259): Poisson on [-1,1]^2 with zero Dirichlet data in the
recombined ultraspherical basis (3.2), solved by the ADI iteration of
Algorithm 2 with the Zolotarev shifts of Theorem 2.1.

This module is a thin ctypes binding of the C ABI in include/fps.h: it
marshals arguments only.  Device memory and the stream come from PyTorch;
every step of the solve runs in the library's HIP kernels.  If libfps.so is
not built, importing works but every call raises RuntimeError.
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["lib", "Plan", "plan", "plan_cylinder", "cylinder_mode_bands", "solve",
           "solve_noalloc", "noalloc_capacity",
           "solve_dirichlet", "solve_adjoint", "solve_fn",
           "adi_native",
           "adi_shifts", "Batch", "batch", "batch_solve", "batch_solve_adjoint", "BatchGraph",
           "FpsError", "LIB_PATH"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfps.so")

FPS_OK, FPS_E_ARG, FPS_E_UNSUPPORTED, FPS_E_NOMEM, FPS_E_HIP, FPS_E_STATE = range(6)
FPS_FP64, FPS_FP32_REFINED = 0, 1
FPS_OUT_CHEB, FPS_OUT_NATIVE = 0, 1
FPS_PLAN_HOST_ONLY = 1
FPS_PLAN_TIGHT_SPECTRUM = 2
FPS_PLAN_CUBE_ZEIG = 4
FPS_PLAN_DIRICHLET = 8

_lib = None


class FpsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fps status {status}: {msg}")
        self.status = status


def lib() -> ctypes.CDLL:
    """The loaded libfps.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run "
                           "`python -m paper_1710_11259_amd.build` first")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
    L.fps_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, i64, ctypes.c_int, dbl,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_uint]
    L.fps_plan_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(i64),
                                ctypes.POINTER(i64)]
    L.fps_plan_create_rect.argtypes = [ctypes.POINTER(vp), i64, ctypes.POINTER(dbl), dbl,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_uint]
    L.fps_plan_shifts.argtypes = [vp, ctypes.POINTER(dbl)]
    L.fps_plan_shift_pairs.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    L.fps_solve_dirichlet.argtypes = [vp, vp, vp, vp, vp, vp]
    L.fps_plan_create_cylinder.argtypes = [ctypes.POINTER(vp), i64, i64, ctypes.c_uint]
    L.fps_cylinder_mode_bands.argtypes = [i64, i64, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    L.fps_plan_refinement.argtypes = [vp, ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_int)]
    L.fps_plan_inner_counts.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.c_int]
    L.fps_plan_rounds.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(dbl),
                                  ctypes.c_int]
    L.fps_plan_slice_counts.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int)]
    L.fps_adi_shifts.argtypes = [dbl, dbl, dbl, dbl, dbl, ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_int), ctypes.POINTER(dbl),
                                 ctypes.POINTER(dbl)]
    for name in ("fps_solve", "fps_solve_adjoint", "fps_adi_native"):
        getattr(L, name).argtypes = [vp, vp, vp, vp, vp]
    L.fps_solve_noalloc.argtypes = [vp, vp, vp, vp]
    L.fps_noalloc_capacity.argtypes = []
    L.fps_probe_stream.argtypes = [vp, vp, vp, i64, vp]
    L.fps_noalloc_capacity.restype = i64
    L.fps_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(i64), dbl, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_uint]
    L.fps_batch_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                 ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_int)]
    L.fps_batch_solve.argtypes = [vp, vp, vp, vp, vp]
    L.fps_batch_solve_adjoint.argtypes = [vp, vp, vp, vp, vp]
    L.fps_batch_destroy.argtypes = [vp]
    L.fps_batch_destroy.restype = None
    L.fps_plan_set_sweep_timing.argtypes = [vp, ctypes.c_int]
    L.fps_plan_sweep_time.argtypes = [vp, ctypes.POINTER(dbl), i64, ctypes.POINTER(i64)]
    L.fps_plan_set_sweep_timing.restype = ctypes.c_int
    L.fps_plan_sweep_time.restype = ctypes.c_int
    L.fps_plan_destroy.argtypes = [vp]
    L.fps_plan_destroy.restype = None
    L.fps_status_string.argtypes = [ctypes.c_int]
    L.fps_status_string.restype = ctypes.c_char_p
    L.fps_last_error.restype = ctypes.c_char_p
    L.fps_version.restype = ctypes.c_char_p
    for name in ("fps_plan_create_cylinder", "fps_cylinder_mode_bands",
                 "fps_plan_create", "fps_plan_create_rect", "fps_plan_shift_pairs",
                 "fps_solve_dirichlet",
                 "fps_plan_create", "fps_plan_info", "fps_plan_shifts", "fps_plan_refinement",
                 "fps_plan_inner_counts", "fps_plan_slice_counts", "fps_plan_rounds",
                 "fps_adi_shifts", "fps_solve", "fps_solve_adjoint", "fps_adi_native",
                 "fps_solve_noalloc",
                 "fps_batch_create", "fps_batch_info", "fps_batch_solve",
                 "fps_batch_solve_adjoint"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int) -> None:
    if status != FPS_OK:
        raise FpsError(status, lib().fps_last_error().decode())


def adi_shifts(a: float, b: float, c: float, d: float, tol: float):
    """(p, q) of Theorem 2.1 from the library's host planner (lists)."""
    L = lib()
    J = ctypes.c_int(0)
    st = L.fps_adi_shifts(a, b, c, d, tol, 0, ctypes.byref(J), None, None)
    if st not in (FPS_OK, FPS_E_STATE):
        _check(st)
    p = (ctypes.c_double * J.value)()
    q = (ctypes.c_double * J.value)()
    _check(L.fps_adi_shifts(a, b, c, d, tol, J.value, ctypes.byref(J), p, q))
    return list(p), list(q)


class Plan:
    """Owning wrapper of an fps_plan.  With `box` = (a, b, c, d) the plan is
    a rectangle plan (fps_plan_create_rect, dim 2); `dirichlet` builds the lift
    map that solve_dirichlet needs (FPS_PLAN_DIRICHLET)."""

    def __init__(self, n: int, tol: float = 1e-13, dim: int = 2, precision: str = "fp64",
                 out: str = "cheb", host_only: bool = False, tight: bool = False,
                 zeig: bool = False, box=None, dirichlet: bool = False, n_theta=None):
        prec = {"fp64": FPS_FP64, "fp32_refined": FPS_FP32_REFINED}[precision]
        ob = {"cheb": FPS_OUT_CHEB, "native": FPS_OUT_NATIVE}[out]
        h = ctypes.c_void_p()
        flags = ((FPS_PLAN_HOST_ONLY if host_only else 0) | (FPS_PLAN_TIGHT_SPECTRUM if tight else 0)
                 | (FPS_PLAN_CUBE_ZEIG if zeig else 0) | (FPS_PLAN_DIRICHLET if dirichlet else 0))
        self._h = ctypes.c_void_p()
        self.n_theta = n_theta
        if n_theta is not None:
            _check(lib().fps_plan_create_cylinder(ctypes.byref(h), n, int(n_theta),
                                                  FPS_PLAN_HOST_ONLY if host_only else 0))
            dim = 3
        elif box is not None:
            if dim != 2:
                raise ValueError("a box applies to 2-D plans only")
            b = (ctypes.c_double * 4)(*[float(v) for v in box])
            _check(lib().fps_plan_create_rect(ctypes.byref(h), n, b, tol, prec, ob, flags))
            box = tuple(float(v) for v in box)
        else:
            _check(lib().fps_plan_create(ctypes.byref(h), dim, n, 0, tol, prec, ob, flags))
        self._h = h
        self.n, self.dim, self.tol, self.precision, self.out = n, dim, tol, precision, out
        self.tight, self.zeig, self.box, self.dirichlet = tight, zeig, box, dirichlet
        J, ws, oe = ctypes.c_int(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().fps_plan_info(h, ctypes.byref(J), ctypes.byref(ws), ctypes.byref(oe)))
        self.J, self.workspace_bytes, self.out_entries = J.value, ws.value, oe.value
        r, f = ctypes.c_int(), ctypes.c_int()
        _check(lib().fps_plan_refinement(h, ctypes.byref(r), ctypes.byref(f)))
        self.rounds, self.f32_steps = r.value, f.value

    @property
    def handle(self):
        return self._h

    def shifts(self):
        p = (ctypes.c_double * self.J)()
        _check(lib().fps_plan_shifts(self._h, p))
        return list(p)

    def shift_pairs(self):
        """(p, q) of Theorem 2.1 as the plan's ADI runs them."""
        p = (ctypes.c_double * self.J)()
        q = (ctypes.c_double * self.J)()
        _check(lib().fps_plan_shift_pairs(self._h, p, q))
        return list(p), list(q)

    def slice_counts(self):
        """Cube plans with zeig: ADI steps per z-slice (descending)."""
        k = ctypes.c_int()
        _check(lib().fps_plan_slice_counts(self._h, None, 0, ctypes.byref(k)))
        c = (ctypes.c_int * max(k.value, 1))()
        _check(lib().fps_plan_slice_counts(self._h, c, k.value, ctypes.byref(k)))
        return list(c)[: k.value]

    def round_steps(self):
        """Square and rectangle plans: (steps, inner tolerance) of each
        refinement round (one round for FP64 plans)."""
        st = (ctypes.c_int * self.rounds)()
        tl = (ctypes.c_double * self.rounds)()
        _check(lib().fps_plan_rounds(self._h, st, tl, self.rounds))
        return list(st), list(tl)

    def inner_counts(self):
        """Cube plans: inner ADI steps per outer step."""
        c = (ctypes.c_int * self.J)()
        _check(lib().fps_plan_inner_counts(self._h, c, self.J))
        return list(c)

    def set_sweep_timing(self, capacity: int):
        _check(lib().fps_plan_set_sweep_timing(self._h, capacity))

    def sweep_time(self, cap: int = 1 << 20):
        """Per-launch milliseconds of the timed half-sweeps since the last call
        (half-step 1 and half-step 2 alternate)."""
        buf = (ctypes.c_double * cap)()
        cnt = ctypes.c_int64()
        _check(lib().fps_plan_sweep_time(self._h, buf, cap, ctypes.byref(cnt)))
        return list(buf[: min(cnt.value, cap)])

    def out_shape(self):
        if self.n_theta is not None:
            return (self.n_theta, 2, self.n + 4, self.n + 2)
        e = self.n if self.out == "native" else self.n + 2
        return (e,) * self.dim

    def in_shape(self):
        if self.n_theta is not None:
            return (self.n_theta, 2, self.n, self.n)
        return (self.n,) * self.dim

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().fps_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan(n: int, tol: float = 1e-13, dim: int = 2, precision: str = "fp64",
         out: str = "cheb", host_only: bool = False, tight: bool = False,
         zeig: bool = False, box=None, dirichlet: bool = False) -> Plan:
    return Plan(n, tol, dim, precision, out, host_only, tight, zeig, box, dirichlet)


def plan_cylinder(n: int, n_theta: int, host_only: bool = False) -> Plan:
    """Cylinder plan (fps_plan_create_cylinder): solve() then takes the
    doubled-up right-hand side as split complex [n_theta][2][n][n]."""
    return Plan(n, host_only=host_only, n_theta=n_theta)


def cylinder_mode_bands(n: int, k: int):
    """(P, Q) bands of mode k's r-operators, each (n/2, 5), offsets -2..2."""
    import numpy as np
    P = np.zeros((n // 2, 5))
    Q = np.zeros((n // 2, 5))
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().fps_cylinder_mode_bands(n, k, P.ctypes.data_as(dp), Q.ctypes.data_as(dp)))
    return P, Q


def _stream_ptr(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def workspace(p: Plan, device="cuda"):
    import torch
    return torch.empty(max(p.workspace_bytes, 256), dtype=torch.uint8, device=device)


def solve(p: Plan, F, out=None, ws=None):
    """U = solve(F) for a float64 CUDA tensor F of shape (n,)*dim."""
    import torch
    if F.dtype != torch.float64 or not F.is_cuda or not F.is_contiguous():
        raise ValueError("F must be a contiguous float64 tensor on the GPU")
    if tuple(F.shape) != p.in_shape():
        raise ValueError(f"F must have shape {p.in_shape()}")
    if out is None:
        out = torch.empty(p.out_shape(), dtype=torch.float64, device=F.device)
    if ws is None:
        ws = workspace(p, F.device)
    _check(lib().fps_solve(p.handle, ctypes.c_void_p(F.data_ptr()),
                           ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                           _stream_ptr(torch, F.device)))
    return out


def solve_noalloc(p: Plan, F, out=None):
    """solve() with the workspace in the library's static device scratch
    (fps_solve_noalloc): square and rectangle plans whose workspace fits
    noalloc_capacity() bytes.  Calls that overlap on one GPU race."""
    import torch
    if F.dtype != torch.float64 or not F.is_cuda or not F.is_contiguous():
        raise ValueError("F must be a contiguous float64 tensor on the GPU")
    if tuple(F.shape) != p.in_shape():
        raise ValueError(f"F must have shape {p.in_shape()}")
    if out is None:
        out = torch.empty(p.out_shape(), dtype=torch.float64, device=F.device)
    _check(lib().fps_solve_noalloc(p.handle, ctypes.c_void_p(F.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()), _stream_ptr(torch, F.device)))
    return out


def probe_stream(a, b, c):
    """c = a + b over float64 device tensors of one length (the streaming
    pass that measures the achievable HBM rate), on the current stream."""
    import torch
    for t in (a, b, c):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise FpsError("probe_stream takes contiguous float64 device tensors")
    if not (a.numel() == b.numel() == c.numel()):
        raise FpsError("probe_stream: tensors of different lengths")
    _check(lib().fps_probe_stream(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                  ctypes.c_void_p(c.data_ptr()), a.numel(),
                                  _stream_ptr(torch, a.device)))


def noalloc_capacity() -> int:
    """Bytes of the static scratch behind solve_noalloc."""
    return int(lib().fps_noalloc_capacity())


def solve_dirichlet(p: Plan, F, bc, out=None, ws=None):
    """U for f with coefficients F (n x n) and Dirichlet traces bc (4 x (n+2):
    L, R in t, B, T in s), on a square or rectangle plan created with
    dirichlet=True and Chebyshev output."""
    import torch
    for name, t, shape in (("F", F, (p.n, p.n)), ("bc", bc, (4, p.n + 2))):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 tensor on the GPU")
        if tuple(t.shape) != shape:
            raise ValueError(f"{name} must have shape {shape}")
    if out is None:
        out = torch.empty(p.out_shape(), dtype=torch.float64, device=F.device)
    if ws is None:
        ws = workspace(p, F.device)
    _check(lib().fps_solve_dirichlet(p.handle, ctypes.c_void_p(F.data_ptr()),
                                     ctypes.c_void_p(bc.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(ws.data_ptr()),
                                     _stream_ptr(torch, F.device)))
    return out


def solve_adjoint(p: Plan, Ubar, out=None, ws=None):
    """Fbar with <solve(F), Ubar> = <F, Fbar> (the transpose of the solve map)."""
    import torch
    if Ubar.dtype != torch.float64 or not Ubar.is_cuda or not Ubar.is_contiguous():
        raise ValueError("Ubar must be a contiguous float64 tensor on the GPU")
    if tuple(Ubar.shape) != p.out_shape():
        raise ValueError(f"Ubar must have shape {p.out_shape()}")
    if out is None:
        out = torch.empty((p.n,) * p.dim, dtype=torch.float64, device=Ubar.device)
    if ws is None:
        ws = workspace(p, Ubar.device)
    _check(lib().fps_solve_adjoint(p.handle, ctypes.c_void_p(Ubar.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(ws.data_ptr()),
                                   _stream_ptr(torch, Ubar.device)))
    return out


def _solve_fn_class():
    import torch

    def batch_of(plan, count):
        # a batch of `count` problems of the plan's size (square FP64 plans),
        # built once per count and kept on the plan
        if (plan.dim != 2 or plan.box is not None or plan.dirichlet or plan.n_theta is not None
                or plan.precision != "fp64" or count < 2):
            return None
        cache = plan.__dict__.setdefault("_batches", {})
        if count not in cache:
            cache[count] = Batch([plan.n] * count, tol=plan.tol, out=plan.out, tight=plan.tight)
        return cache[count]

    class SolveFn(torch.autograd.Function):
        """Differentiable square solve.  forward: U = solve(F) for F of shape
        (n, n) or (batch, n, n); backward: the adjoint solve (same ADI sweeps
        between transposed coefficient maps), nothing stored from the forward
        pass because the map is linear in F.  A batch of square FP64 problems
        runs as one fps_batch (sweeps of all problems in one launch per
        half-step, forward and backward); its results equal the per-problem
        solves."""

        @staticmethod
        def forward(ctx, F, plan):
            ctx.plan = plan
            Fc = F.contiguous()
            if Fc.dim() == 2:
                return solve(plan, Fc, ws=workspace(plan, F.device))
            b = batch_of(plan, Fc.shape[0])
            if b is not None:
                e = plan.n if plan.out == "native" else plan.n + 2
                ws = torch.empty(max(b.workspace_bytes, 256), dtype=torch.uint8, device=F.device)
                return batch_solve(b, Fc.reshape(-1), ws=ws).view(Fc.shape[0], e, e)
            ws = workspace(plan, F.device)
            return torch.stack([solve(plan, Fc[i], ws=ws) for i in range(Fc.shape[0])])

        @staticmethod
        def backward(ctx, Ubar):
            plan = ctx.plan
            Uc = Ubar.contiguous()
            if Uc.dim() == 2:
                return solve_adjoint(plan, Uc, ws=workspace(plan, Ubar.device)), None
            b = batch_of(plan, Uc.shape[0])
            if b is not None:
                ws = torch.empty(max(b.workspace_bytes, 256), dtype=torch.uint8, device=Ubar.device)
                Fb = batch_solve_adjoint(b, Uc.reshape(-1), ws=ws)
                return Fb.view(Uc.shape[0], plan.n, plan.n), None
            ws = workspace(plan, Ubar.device)
            return torch.stack([solve_adjoint(plan, Uc[i], ws=ws)
                                for i in range(Uc.shape[0])]), None

    return SolveFn


def solve_fn(F, plan: Plan):
    """Autograd entry point: SolveFn.apply(F, plan)."""
    global _SolveFn
    try:
        cls = _SolveFn
    except NameError:
        cls = _SolveFn = _solve_fn_class()
    return cls.apply(F, plan)


def adi_native(p: Plan, G, out=None, ws=None):
    """Y_J of Algorithm 2 for A~ Y + Y A~ = G (natural order, n x n); for a
    rectangle plan sx2 A~ Y + sy2 Y A~ = G."""
    import torch
    if G.dtype != torch.float64 or not G.is_cuda or not G.is_contiguous():
        raise ValueError("G must be a contiguous float64 tensor on the GPU")
    if tuple(G.shape) != (p.n, p.n):
        raise ValueError("G must be n x n")
    if out is None:
        out = torch.empty((p.n, p.n), dtype=torch.float64, device=G.device)
    if ws is None:
        ws = workspace(p, G.device)
    _check(lib().fps_adi_native(p.handle, ctypes.c_void_p(G.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                _stream_ptr(torch, G.device)))
    return out


class Batch:
    """Owning wrapper of an fps_batch: independent square solves of sizes
    ns (packed back to back), ADI half-sweeps of all problems in one launch
    per half-step."""

    def __init__(self, ns, tol: float = 1e-13, precision: str = "fp64", out: str = "cheb",
                 host_only: bool = False, tight: bool = False):
        prec = {"fp64": FPS_FP64, "fp32_refined": FPS_FP32_REFINED}[precision]
        ob = {"cheb": FPS_OUT_CHEB, "native": FPS_OUT_NATIVE}[out]
        self.ns = [int(v) for v in ns]
        arr = (ctypes.c_int64 * len(self.ns))(*self.ns)
        h = ctypes.c_void_p()
        flags = (FPS_PLAN_HOST_ONLY if host_only else 0) | (FPS_PLAN_TIGHT_SPECTRUM if tight else 0)
        _check(lib().fps_batch_create(ctypes.byref(h), 2, len(self.ns), arr, tol, prec, ob, flags))
        self._h = h
        self.tol, self.precision, self.out = tol, precision, out
        ws, ie, oe, J = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int()
        _check(lib().fps_batch_info(h, ctypes.byref(ws), ctypes.byref(ie), ctypes.byref(oe),
                                    ctypes.byref(J)))
        self.workspace_bytes, self.in_entries, self.out_entries = ws.value, ie.value, oe.value
        self.max_J = J.value
        e = [v if out == "native" else v + 2 for v in self.ns]
        self.in_offsets = [0]
        self.out_offsets = [0]
        for v, ev in zip(self.ns, e):
            self.in_offsets.append(self.in_offsets[-1] + v * v)
            self.out_offsets.append(self.out_offsets[-1] + ev * ev)

    @property
    def handle(self):
        return self._h

    def pack(self, Fs, device="cuda"):
        """Pack a list of n_b x n_b float64 arrays/tensors into one device tensor."""
        import torch
        parts = [torch.as_tensor(F, dtype=torch.float64).reshape(-1) for F in Fs]
        return torch.cat(parts).to(device).contiguous()

    def unpack(self, U):
        """Views of the packed output as a list of square tensors."""
        e = [v if self.out == "native" else v + 2 for v in self.ns]
        return [U[self.out_offsets[b]:self.out_offsets[b + 1]].view(e[b], e[b])
                for b in range(len(self.ns))]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().fps_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch(ns, tol: float = 1e-13, precision: str = "fp64", out: str = "cheb",
          host_only: bool = False, tight: bool = False) -> Batch:
    return Batch(ns, tol, precision, out, host_only, tight)


def batch_solve(b: Batch, F, out=None, ws=None):
    """Packed U for the packed float64 CUDA tensor F (see Batch.pack)."""
    import torch
    if F.dtype != torch.float64 or not F.is_cuda or not F.is_contiguous():
        raise ValueError("F must be a contiguous float64 tensor on the GPU")
    if F.numel() != b.in_entries:
        raise ValueError(f"F must hold {b.in_entries} entries")
    if out is None:
        out = torch.empty(b.out_entries, dtype=torch.float64, device=F.device)
    if out.numel() != b.out_entries or not out.is_contiguous():
        raise ValueError(f"out must be contiguous with {b.out_entries} entries")
    if ws is None:
        ws = torch.empty(max(b.workspace_bytes, 256), dtype=torch.uint8, device=F.device)
    _check(lib().fps_batch_solve(b.handle, ctypes.c_void_p(F.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                 _stream_ptr(torch, F.device)))
    return out


def batch_solve_adjoint(b: Batch, Ubar, out=None, ws=None):
    """Packed Fbar (the VJP of batch_solve) for the packed float64 CUDA
    tensor Ubar in the batch's output layout."""
    import torch
    if Ubar.dtype != torch.float64 or not Ubar.is_cuda or not Ubar.is_contiguous():
        raise ValueError("Ubar must be a contiguous float64 tensor on the GPU")
    if Ubar.numel() != b.out_entries:
        raise ValueError(f"Ubar must hold {b.out_entries} entries")
    if out is None:
        out = torch.empty(b.in_entries, dtype=torch.float64, device=Ubar.device)
    if out.numel() != b.in_entries or not out.is_contiguous():
        raise ValueError(f"out must be contiguous with {b.in_entries} entries")
    if ws is None:
        ws = torch.empty(max(b.workspace_bytes, 256), dtype=torch.uint8, device=Ubar.device)
    _check(lib().fps_batch_solve_adjoint(b.handle, ctypes.c_void_p(Ubar.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(ws.data_ptr()),
                                         _stream_ptr(torch, Ubar.device)))
    return out


class BatchGraph:
    """A batched solve captured once into a HIP graph (through torch's graph
    capture) and replayed with one launch.  F, U and the workspace are fixed
    device buffers: write new inputs into `self.F` before `replay()`."""

    def __init__(self, b: Batch, device="cuda"):
        import torch
        self.batch = b
        self.F = torch.zeros(b.in_entries, dtype=torch.float64, device=device)
        self.U = torch.empty(b.out_entries, dtype=torch.float64, device=device)
        self.ws = torch.empty(max(b.workspace_bytes, 256), dtype=torch.uint8, device=device)
        side = torch.cuda.Stream(device)
        side.wait_stream(torch.cuda.current_stream(device))
        with torch.cuda.stream(side):  # one eager run before capture
            batch_solve(b, self.F, out=self.U, ws=self.ws)
        torch.cuda.current_stream(device).wait_stream(side)
        torch.cuda.synchronize(device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            batch_solve(b, self.F, out=self.U, ws=self.ws)
        torch.cuda.synchronize(device)

    def replay(self):
        self.graph.replay()
        return self.U


class SolveGraph:
    """One solve of plan `p` (any shape: square, rectangle, cube, cylinder)
    captured into a HIP graph and replayed with one launch.  fps_solve
    enqueues kernels only, so the capture holds no memset or memcpy nodes.
    F, U and the workspace are fixed device buffers: write new inputs into
    `self.F` before `replay()`.  Capture with the plan's sweep timing off
    (set_sweep_timing(0)): timed launches record events."""

    def __init__(self, p: Plan, device="cuda"):
        import torch
        self.plan = p
        self.F = torch.zeros(p.in_shape(), dtype=torch.float64, device=device)
        self.U = torch.empty(p.out_shape(), dtype=torch.float64, device=device)
        self.ws = workspace(p, device)
        side = torch.cuda.Stream(device)
        side.wait_stream(torch.cuda.current_stream(device))
        with torch.cuda.stream(side):  # one eager run before capture
            solve(p, self.F, out=self.U, ws=self.ws)
        torch.cuda.current_stream(device).wait_stream(side)
        torch.cuda.synchronize(device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            solve(p, self.F, out=self.U, ws=self.ws)
        torch.cuda.synchronize(device)

    def replay(self):
        self.graph.replay()
        return self.U
