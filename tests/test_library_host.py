"""CPU tests of the product library: ABI exports, host planner against the
oracle, argument validation (no device compute)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1710_11259_amd as fps
from oracle import basis, shifts as oshifts, square

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "fps.h")).read()
    return sorted(set(re.findall(r"\b(fps_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = fps.lib()
    syms = _declared_symbols()
    assert len(syms) >= 10
    for s in syms:
        assert hasattr(L, s), s
    out = subprocess.run(["nm", "-D", "--defined-only", fps.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    for s in syms:
        assert re.search(rf"\bT {s}$", out, re.M), s


def test_version_and_status_strings():
    L = fps.lib()
    assert b"gfx950" in L.fps_version()
    assert L.fps_status_string(0) == b"ok"


@pytest.mark.parametrize("n", [1, 2, 5, 16, 24, 25, 64, 1024, 4096, 10000])
def test_plan_shifts_match_oracle(n):
    p = fps.plan(n, tol=1e-13, host_only=True)
    J, po, _ = oshifts.square_shifts(n, 1e-13)
    assert p.J == J
    # applied in order of increasing |p_j|, the reverse of Theorem 2.1's indexing
    assert np.allclose(p.shifts(), po[::-1], rtol=2e-14, atol=0)


@pytest.mark.parametrize("iv", [(-5.0, -0.5, 0.2, 3.0), (-1.0, -1e-3, 1e-3, 1.0), (-2.0, -1.0, 3.0, 100.0)])
def test_general_interval_shifts_match_oracle(iv):
    p, q = fps.adi_shifts(*iv, 1e-10)
    J, po, qo = oshifts.zolotarev_shifts(*iv, tol=1e-10)
    assert len(p) == J
    assert np.allclose(p, po, rtol=1e-13, atol=1e-15 * max(map(abs, iv)))
    assert np.allclose(q, qo, rtol=1e-13, atol=1e-15 * max(map(abs, iv)))


def test_argument_errors():
    L = fps.lib()
    h = ctypes.c_void_p()
    for args, code in [((2, 0, 0, 1e-13, 0, 0, 1), 1), ((2, 16, 0, 0.0, 0, 0, 1), 1),
                       ((2, 16, 0, 1.0, 0, 0, 1), 1), ((4, 16, 0, 1e-13, 0, 0, 1), 1),
                       ((2, 16, 7, 1e-13, 0, 0, 1), 2), ((2, 16, 0, 1e-13, 9, 0, 1), 1),
                       ((2, 16, 0, 1e-13, 0, 5, 1), 1), ((2, 16, 0, 1e-13, 0, 0, 16), 1)]:
        assert L.fps_plan_create(ctypes.byref(h), *args) == code, args
        assert len(L.fps_last_error()) > 0
    J = ctypes.c_int()
    assert L.fps_adi_shifts(1.0, 0.5, 2.0, 3.0, 1e-8, 0, ctypes.byref(J), None, None) == 1
    assert L.fps_adi_shifts(-1.0, -0.5, 2.0, 3.0, 1e-8, 0, ctypes.byref(J), None, None) == 5
    assert J.value > 0
    # solve on a host-only plan / null plan
    p = fps.plan(16, host_only=True)
    assert L.fps_solve(p.handle, None, None, None, None) == 5
    assert L.fps_solve(None, None, None, None, None) == 5
    assert L.fps_plan_info(None, None, None, None) == 5


def test_workspace_and_extent_queries():
    p = fps.plan(100, host_only=True)
    assert p.out_entries == 102 * 102
    assert p.workspace_bytes >= 4 * 128 * 128 * 8
    q = fps.plan(100, out="native", host_only=True)
    assert q.out_entries == 100 * 100


def test_size_limits():
    # square/rectangle plans up to n = 16384 (the register form of the
    # chunk-carry scan), nested cubes to 384, z-eigenbasis cubes to 512
    with pytest.raises(fps.FpsError) as e:
        fps.plan(16385, host_only=True)
    assert e.value.status == fps.FPS_E_UNSUPPORTED
    with pytest.raises(fps.FpsError) as e:
        fps.plan(385, dim=3, host_only=True)
    assert e.value.status == fps.FPS_E_UNSUPPORTED
    with pytest.raises(fps.FpsError) as e:
        fps.plan(513, dim=3, zeig=True, host_only=True)
    assert e.value.status == fps.FPS_E_UNSUPPORTED
    with pytest.raises(fps.FpsError):
        fps.batch([64, 16385], host_only=True)


@pytest.mark.parametrize("n", [64, 512, 4096])
def test_refinement_structure(n):
    # FP64: one round, no float steps.  FP32_REFINED to 1e-13: rounds to
    # 1e-5, 1e-5 and a last one to 0.1 * 1e-13 / 1e-10 = 1e-4, every step
    # storing in float, each round's J from (2.9) and its shifts applied in
    # order of increasing |p_j|.
    d = fps.plan(n, tol=1e-13, host_only=True)
    assert (d.rounds, d.f32_steps) == (1, 0)
    assert d.round_steps() == ([d.J], [1e-13])
    r = fps.plan(n, tol=1e-13, precision="fp32_refined", host_only=True)
    steps, tols = r.round_steps()
    assert r.rounds == 3
    np.testing.assert_allclose(tols, [1e-5, 1e-5, 1e-4], rtol=1e-12)
    for J, t in zip(steps, tols):
        assert J == oshifts.square_shifts(n, t)[0]
    assert r.f32_steps == sum(steps)
    _, p, _ = oshifts.square_shifts(n, 1e-5)
    assert r.J == steps[0] == len(p)
    np.testing.assert_allclose(r.shifts(), p[::-1], rtol=2e-14)
    assert np.all(np.diff(np.abs(r.shifts())) > 0)
    assert r.workspace_bytes > d.workspace_bytes
    # looser targets take fewer rounds
    r10 = fps.plan(n, tol=1e-10, precision="fp32_refined", host_only=True)
    np.testing.assert_allclose(r10.round_steps()[1], [1e-5, 1e-6], rtol=1e-12)
    r3 = fps.plan(n, tol=1e-3, precision="fp32_refined", host_only=True)
    np.testing.assert_allclose(r3.round_steps()[1], [1e-3], rtol=1e-12)


@pytest.mark.parametrize("n", [1, 16, 256])
def test_cube_plan_outer_shifts_match_oracle(n):
    from oracle import cube
    p = fps.plan(n, tol=1e-13, dim=3, host_only=True)
    J, po, _ = cube.kform_outer_shifts(n, 1e-13)
    assert p.J == J
    np.testing.assert_allclose(p.shifts(), po, rtol=1e-12)
    assert p.out_entries == (n + 2) ** 3
    assert fps.plan(n, dim=3, out="native", host_only=True).out_entries == n ** 3
    # inner counts: (2.9) for the symmetric inner intervals at tol / 10
    q = cube.kform_outer_shifts(n, 1e-13)[2]
    want = [cube.kform_inner_shifts(n, qi, 1e-14)[0] for qi in q]
    assert p.inner_counts() == want


def test_cube_plan_refined_needs_zeig():
    # the nested method has no refined form; the z-eigenbasis method does
    with pytest.raises(fps.FpsError) as e:
        fps.plan(8, dim=3, precision="fp32_refined", host_only=True)
    assert e.value.status == fps.FPS_E_UNSUPPORTED
    p = fps.plan(64, tol=1e-13, dim=3, zeig=True, tight=True, precision="fp32_refined",
                 host_only=True)
    steps, tols = p.round_steps()
    np.testing.assert_allclose(tols, [1e-5, 1e-5, 1e-4], rtol=1e-12)
    assert p.rounds == 3 and p.f32_steps == sum(steps)
    # slices sorted by |mu| descending: step counts of round 0 non-increasing
    c = p.slice_counts()
    assert len(c) == 64 and all(a >= b for a, b in zip(c, c[1:])) and c[0] == steps[0]


def test_batch_queries_and_errors():
    ns = [32, 64, 544, 32, 1, 129]
    b = fps.batch(ns, host_only=True)
    assert b.in_entries == sum(n * n for n in ns)
    assert b.out_entries == sum((n + 2) ** 2 for n in ns)
    plans = {n: fps.plan(n, host_only=True) for n in set(ns)}
    assert b.max_J == max(p.J for p in plans.values())
    assert b.workspace_bytes == sum((plans[n].workspace_bytes + 255) // 256 * 256 for n in ns)
    bn = fps.batch(ns, out="native", host_only=True)
    assert bn.out_entries == sum(n * n for n in ns)
    L = fps.lib()
    h = ctypes.c_void_p()
    arr = (ctypes.c_int64 * 2)(4, 0)
    assert L.fps_batch_create(ctypes.byref(h), 2, 2, arr, 1e-13, 0, 0, 1) == fps.FPS_E_ARG
    arr = (ctypes.c_int64 * 1)(4)
    assert L.fps_batch_create(ctypes.byref(h), 2, 0, arr, 1e-13, 0, 0, 1) == fps.FPS_E_ARG
    assert L.fps_batch_create(ctypes.byref(h), 3, 1, arr, 1e-13, 0, 0, 1) == fps.FPS_E_UNSUPPORTED
    assert L.fps_batch_create(ctypes.byref(h), 2, 1, arr, 2.0, 0, 0, 1) == fps.FPS_E_ARG
    assert L.fps_batch_solve(None, None, None, None, None) == fps.FPS_E_STATE
    hb = fps.batch([8], host_only=True)
    assert L.fps_batch_solve(hb.handle, None, None, None, None) == fps.FPS_E_STATE
    assert L.fps_batch_solve_adjoint(None, None, None, None, None) == fps.FPS_E_STATE
    assert L.fps_batch_solve_adjoint(hb.handle, None, None, None, None) == fps.FPS_E_STATE


# --- host planner internals through a g++-built shim -----------------------

@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    d = tmp_path_factory.mktemp("shim")
    so = str(d / "libshim.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", so,
                    os.path.join(ROOT, "tests", "planner_shim.cpp"),
                    os.path.join(ROOT, "paper_1710_11259_amd", "csrc", "planner.cpp")],
                   check=True)
    L = ctypes.CDLL(so)
    P = ctypes.POINTER(ctypes.c_double)
    L.shim_layout.argtypes = [ctypes.c_longlong, ctypes.POINTER(ctypes.c_longlong)]
    L.shim_tables.argtypes = [ctypes.c_longlong, ctypes.c_int, P, P, P]
    L.shim_conversions.argtypes = [ctypes.c_longlong, P, P, P, P]
    L.shim_dn.argtypes = [ctypes.c_double, ctypes.c_int, P]
    L.shim_extremes.argtypes = [ctypes.c_longlong, P]
    L.shim_lift_map.argtypes = [ctypes.c_longlong, P, P]
    return L


def _layout(shim, n):
    v = (ctypes.c_longlong * 14)()
    shim.shim_layout(n, v)
    keys = ["m0", "m1", "mp0", "mp1", "npad", "nc0", "nc1", "ncmax", "mstride", "mo0", "mo1",
            "seg", "waves", "chunk"]
    return dict(zip(keys, list(v)))


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@pytest.mark.parametrize("alpha", [30.0, 480.0, 7680.0, 1.2e5, 2e6, 9.9e6, 1e7, 3.1e9, 4.8e13,
                                   7.7e17, 1e20])
def test_complementary_parameter_dn_matches_exact(shim, alpha):
    # K and dn from Carlson's R_F and Newton inversion in m1 = 1/alpha^2, for
    # every alpha (the square enclosure at n = 10^4 reaches alpha ~ 1e18)
    J = 40
    dn = np.zeros(J)
    shim.shim_dn(alpha, J, _ptr(dn))
    assert np.allclose(dn, oshifts.exact_dn(alpha, J), rtol=1e-14)


@pytest.mark.parametrize("delta", [1e-9, 1e-14, 1e-20])
def test_library_shifts_large_alpha_match_exact(delta):
    # symmetric intervals [-1, -delta], [delta, 1]: p_j = -dn_j, so the
    # library's shifts pin its dn at the huge alpha of tiny delta
    p, q = fps.adi_shifts(-1.0, -delta, delta, 1.0, 1e-10)
    g = oshifts.cross_ratio(-1.0, -delta, delta, 1.0)
    alpha = -1.0 + 2.0 * g + 2.0 * np.sqrt(g * g - g)
    assert alpha > 1e8
    np.testing.assert_allclose(-np.array(p), oshifts.exact_dn(alpha, len(p)), rtol=1e-13)
    np.testing.assert_allclose(q, -np.array(p), rtol=0, atol=0)


def test_elem_launch_cap(shim):
    # a 1-D grid of 256-thread workgroups holds at most (2^32 - 1) / 256
    shim.shim_elem_launch_fits.argtypes = [ctypes.c_longlong]
    cap = (2 ** 32 - 1) // 256
    assert shim.shim_elem_launch_fits(cap) == 1
    assert shim.shim_elem_launch_fits(cap + 1) == 0
    assert shim.shim_elem_launch_fits(1 << 25) == 0


def _emulate_partitioned_solve(T, C, lay, s, r):
    """Two-level partitioned Thomas with the planner's tables (kernel algorithm)."""
    ms, seg, W, CH = lay["mstride"], lay["seg"], lay["waves"], lay["chunk"]
    l, ib, u, F1, Bk1, BF2, Bk2 = (T[k] for k in range(7))
    nc = lay["nc%d" % s]
    rr = np.zeros(ms)
    rr[: len(r)] = r
    xloc = np.zeros(ms)
    ylast = np.zeros(nc)
    xfirst = np.zeros(nc)
    for c in range(nc):
        ys, xs = [], []
        for w in range(W):
            k0 = c * CH + w * seg
            y = np.zeros(seg)
            carry = 0.0
            for i in range(seg):
                y[i] = rr[k0 + i] - l[k0 + i] * carry
                carry = y[i]
            ys.append(y)
        cf = 0.0
        for w in range(W):
            k0 = c * CH + w * seg
            ys[w] = ys[w] + F1[k0: k0 + seg] * cf
            cf = ys[w][-1]
        for w in range(W):
            k0 = c * CH + w * seg
            x = np.zeros(seg)
            xn = 0.0
            for i in range(seg - 1, -1, -1):
                x[i] = ys[w][i] * ib[k0 + i] - u[k0 + i] * xn
                xn = x[i]
            xs.append(x)
        cb = 0.0
        for w in range(W - 1, -1, -1):
            k0 = c * CH + w * seg
            xs[w] = xs[w] + Bk1[k0: k0 + seg] * cb
            cb = xs[w][0]
        xloc[c * CH:(c + 1) * CH] = np.concatenate(xs)
        ylast[c] = ys[-1][-1]
        xfirst[c] = xs[0][0]
    F2last, BF2first, Bk2first = C
    cfv = np.zeros(nc)
    for c in range(1, nc):
        cfv[c] = ylast[c - 1] + F2last[c - 1] * cfv[c - 1]
    cbv = np.zeros(nc)
    for c in range(nc - 2, -1, -1):
        cbv[c] = xfirst[c + 1] + BF2first[c + 1] * cfv[c + 1] + Bk2first[c + 1] * cbv[c + 1]
    x = xloc.copy()
    for c in range(nc):
        sl = slice(c * CH, (c + 1) * CH)
        x[sl] += cfv[c] * BF2[sl] + cbv[c] * Bk2[sl]
    return x


@pytest.mark.parametrize("n", [3, 130, 700, 1300])
def test_sweep_tables_reproduce_shifted_solves(shim, n):
    lay = _layout(shim, n)
    J, p, _ = oshifts.square_shifts(n, 1e-13)
    sel = [0, J // 2, J - 1]
    pv = np.ascontiguousarray(p[sel])
    ms, nc = lay["mstride"], lay["ncmax"]
    pos = np.zeros(len(sel) * 2 * 7 * ms)
    ch = np.zeros(len(sel) * 2 * 3 * nc)
    shim.shim_tables(n, len(sel), _ptr(pv), _ptr(pos), _ptr(ch))
    pos = pos.reshape(len(sel), 2, 7, ms)
    ch = ch.reshape(len(sel), 2, 3, nc)
    A = square.atilde_dense(n)
    rng = np.random.default_rng(n)
    for jj, pj in enumerate(pv):
        for s in (0, 1):
            idx = np.arange(s, n, 2)
            if idx.size == 0:
                continue
            Tm = A[np.ix_(idx, idx)] + pj * np.eye(idx.size)
            r = rng.standard_normal(idx.size)
            xr = np.linalg.solve(Tm, r)
            x = _emulate_partitioned_solve(pos[jj, s], ch[jj, s], lay, s, r)
            assert np.linalg.norm(x[: idx.size] - xr) <= 1e-10 * np.linalg.norm(xr)
            assert np.all(x[idx.size:] == 0)


@pytest.mark.parametrize("n", [1, 2, 7, 40, 301])
def test_conversion_maps_match_oracle(shim, n):
    lay = _layout(shim, n)
    m, mo = (lay["m0"], lay["m1"]), (lay["mo0"], lay["mo1"])
    R = [np.zeros(m[s] * m[s]) for s in (0, 1)]
    P = [np.zeros(mo[s] * m[s]) for s in (0, 1)]
    shim.shim_conversions(n, _ptr(R[0]), _ptr(R[1]), _ptr(P[0]), _ptr(P[1]))
    Ro = basis.cheb_to_ct(n)
    Po = basis.recombined_to_cheb(n)
    sinv = 1.0 / square.s_diag(n)
    for s in (0, 1):
        if m[s] == 0:
            continue
        idx = np.arange(s, n, 2)
        oidx = np.arange(s, n + 2, 2)
        Rref = (sinv[:, None] * Ro)[np.ix_(idx, idx)]
        Pref = (Po * sinv[None, :])[np.ix_(oidx, idx)]
        assert np.abs(R[s].reshape(m[s], m[s]) - Rref).max() < 1e-13 * max(1, np.abs(Rref).max())
        assert np.abs(P[s].reshape(mo[s], m[s]) - Pref).max() < 1e-13 * max(1, np.abs(Pref).max())


@pytest.mark.parametrize("n", [3, 33, 130, 255, 256])
def test_chunk_tables_reproduce_shifted_solves(shim, n):
    # The LDS-resident slice kernel's algorithm: every 16-position chunk of a
    # parity chain solved with zero carries (whole-chain factors l, ib, u),
    # then the chunk-level recurrences with F2last, BF2first, Bk2first and the
    # carries added through BF2, Bk2 -- against a dense solve of the shifted
    # parity block of the oracle's A~.
    shim.shim_chunk_tables.argtypes = [ctypes.c_longlong, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_double), ctypes.c_longlong,
                                       ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]
    CH = 16
    lay = _layout(shim, n)
    ms, nc = lay["mstride"], lay["ncmax"]
    J, p, _ = oshifts.square_shifts(n, 1e-13)
    sel = [0, J // 2, J - 1]
    pv = np.ascontiguousarray(p[sel])
    pos = np.zeros(len(sel) * 2 * 7 * ms)
    ch0 = np.zeros(len(sel) * 2 * 3 * nc)
    shim.shim_tables(n, len(sel), _ptr(pv), _ptr(pos), _ptr(ch0))
    pos = pos.reshape(len(sel), 2, 7, ms)
    nq = ms // CH
    t32 = np.zeros(len(sel) * 2 * 2 * ms)
    c32 = np.zeros(len(sel) * 2 * 3 * nq)
    shim.shim_chunk_tables(n, len(sel), _ptr(pv), CH, _ptr(t32), _ptr(c32))
    t32 = t32.reshape(len(sel), 2, 2, ms)
    c32 = c32.reshape(len(sel), 2, 3, nq)
    A = square.atilde_dense(n)
    rng = np.random.default_rng(n + 1)
    for jj, pj in enumerate(pv):
        for s in (0, 1):
            idx = np.arange(s, n, 2)
            m = idx.size
            if m == 0:
                continue
            l, ib, u = pos[jj, s, 0], pos[jj, s, 1], pos[jj, s, 2]
            BF2, Bk2 = t32[jj, s]
            F2last, BF2first, Bk2first = c32[jj, s]
            r = rng.standard_normal(m)
            nq_s = (m + CH - 1) // CH
            x = np.zeros(m)
            ylast, xfirst = np.zeros(nq_s), np.zeros(nq_s)
            for c in range(nq_s):
                k0, k1 = c * CH, min(m, (c + 1) * CH)
                y = np.zeros(k1 - k0)
                yp = 0.0
                for k in range(k0, k1):
                    y[k - k0] = r[k] - l[k] * yp
                    yp = y[k - k0]
                xn = 0.0
                for k in range(k1 - 1, k0 - 1, -1):
                    x[k] = y[k - k0] * ib[k] - u[k] * xn
                    xn = x[k]
                ylast[c], xfirst[c] = yp, x[k0]
            cf, cb = np.zeros(nq_s), np.zeros(nq_s)
            for c in range(1, nq_s):
                cf[c] = F2last[c - 1] * cf[c - 1] + ylast[c - 1]
            for c in range(nq_s - 2, -1, -1):
                cb[c] = Bk2first[c + 1] * cb[c + 1] + xfirst[c + 1] + BF2first[c + 1] * cf[c + 1]
            for c in range(nq_s):
                k0, k1 = c * CH, min(m, (c + 1) * CH)
                x[k0:k1] += cf[c] * BF2[k0:k1] + cb[c] * Bk2[k0:k1]
            xr = np.linalg.solve(A[np.ix_(idx, idx)] + pj * np.eye(m), r)
            assert np.linalg.norm(x - xr) <= 1e-10 * np.linalg.norm(xr), (n, jj, s)


@pytest.mark.parametrize("n", [130, 1300, 4096])
def test_carry_combinations_match_recurrence(shim, n):
    shim.shim_comb.argtypes = [ctypes.c_longlong, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_double)]
    lay = _layout(shim, n)
    J, p, _ = oshifts.square_shifts(n, 1e-13)
    pv = np.ascontiguousarray(p[[0, J // 2, J - 1]])
    ms, nc = lay["mstride"], lay["ncmax"]
    pos = np.zeros(3 * 2 * 7 * ms)
    ch = np.zeros(3 * 2 * 3 * nc)
    comb = np.zeros(3 * 2 * nc * nc * 3)
    shim.shim_tables(n, 3, _ptr(pv), _ptr(pos), _ptr(ch))
    shim.shim_comb(n, 3, _ptr(pv), _ptr(comb))
    ch = ch.reshape(3, 2, 3, nc)
    comb = comb.reshape(3, 2, nc, nc, 3)
    rng = np.random.default_rng(0)
    for jj in range(3):
        for s in (0, 1):
            ncs = lay["nc%d" % s]
            yl, xf = rng.standard_normal(ncs), rng.standard_normal(ncs)
            F2last, BF2first, Bk2first = ch[jj, s]
            cf = np.zeros(ncs)
            for c in range(1, ncs):
                cf[c] = yl[c - 1] + F2last[c - 1] * cf[c - 1]
            cb = np.zeros(ncs)
            for c in range(ncs - 2, -1, -1):
                cb[c] = xf[c + 1] + BF2first[c + 1] * cf[c + 1] + Bk2first[c + 1] * cb[c + 1]
            W = comb[jj, s, :ncs, :ncs]
            assert np.allclose(W[..., 0] @ yl, cf, rtol=1e-13, atol=1e-13)
            assert np.allclose(W[..., 1] @ yl + W[..., 2] @ xf, cb, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("n", [1, 2, 3, 17, 64, 301, 1024])
def test_extreme_eigenvalues_match_lapack(shim, n):
    # Sturm bisection in the planner against LAPACK (the oracle's parity
    # eigen-decomposition); the largest eigenvalue is O(n^-4), so compare
    # relatively.
    out = (ctypes.c_double * 2)()
    shim.shim_extremes(n, out)
    lam, _ = square.atilde_eig(n)
    assert out[0] == pytest.approx(lam.min(), rel=1e-12)
    assert out[1] == pytest.approx(lam.max(), rel=1e-9)


@pytest.mark.parametrize("n", [64, 1024, 4096])
def test_tight_spectrum_plan_counts(n):
    # J from (2.9) on the computed spectrum widened by 1e-6 (the enclosure the
    # flag documents); the counts agree with those of the exact eigenvalues.
    lam, _ = square.atilde_eig(n) if n <= 1024 else (None, None)
    p = fps.plan(n, tol=1e-13, host_only=True, tight=True)
    d = fps.plan(n, tol=1e-13, host_only=True)
    assert p.J < d.J
    if lam is not None:
        a, b = lam.min() * (1 + 1e-6), lam.max() * (1 - 1e-6)
        assert p.J == oshifts.iteration_count(a, b, -b, -a, 1e-13)
        J, po, _ = oshifts.zolotarev_shifts(a, b, -b, -a, tol=1e-13)
        np.testing.assert_allclose(p.shifts(), po[::-1], rtol=1e-8)
    expected = {64: 44, 1024: 78, 4096: 96}
    assert p.J == expected[n]


@pytest.mark.parametrize("n", [1, 2, 7, 40, 257])
def test_tridiagonal_eigensolver_matches_lapack(shim, n):
    # Planner's implicit-QR eigen-decomposition of each parity block of A~:
    # eigenvalues against LAPACK (relative, they span O(n^-4) .. 0.4), and
    # an orthonormal eigenbasis that diagonalizes the block.
    A = square.atilde_dense(n)
    for s in (0, 1):
        m = (n - s + 1) // 2
        if m == 0:
            continue
        lam = (ctypes.c_double * m)()
        Q = (ctypes.c_double * (m * m))()
        shim.shim_atilde_eigen.argtypes = [ctypes.c_longlong, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double)]
        assert shim.shim_atilde_eigen(n, s, lam, Q) == 1
        lam = np.array(lam)
        Q = np.array(Q).reshape(m, m)
        B = A[s::2, s::2]
        ref = np.linalg.eigvalsh(B)
        np.testing.assert_allclose(lam, ref, rtol=1e-10, atol=0)
        assert np.abs(Q.T @ Q - np.eye(m)).max() < 1e-14
        assert np.abs(Q.T @ B @ Q - np.diag(lam)).max() < 1e-15


@pytest.mark.parametrize("n,tight", [(1, False), (5, True), (16, False), (64, True)])
def test_zeig_cube_plan_slice_counts_match_oracle(n, tight):
    # One Algorithm 2 per z-slice, J from (2.9) on the slice intervals of the
    # oracle (eigenvalues from the planner's own eigen-decomposition).
    from oracle import cube
    p = fps.plan(n, tol=1e-13, dim=3, host_only=True, tight=tight, zeig=True)
    lam, _ = square.atilde_eig(n)
    if tight:
        lmin, lmax = lam.min() * (1 + 1e-6), lam.max() * (1 - 1e-6)
    else:
        lmin, lmax = -1.0, -1.0 / (30.0 * n ** 4)
    want = sorted((oshifts.iteration_count(*cube.zeig_slice_intervals(n, mu, lmin, lmax), 1e-13)
                   for mu in lam), reverse=True)
    assert p.slice_counts() == want
    assert p.J == want[0]
    with pytest.raises(fps.FpsError):
        p.inner_counts()


RECT_BOXES = [(0.0, 2.5, -1.0, 0.25), (0.0, 10.0, 0.0, 1.0), (-3.0, 3.0, -3.0, 3.0)]


@pytest.mark.parametrize("box", RECT_BOXES)
@pytest.mark.parametrize("n", [1, 5, 64, 4096])
def test_rect_plan_shifts_match_oracle(n, box):
    from oracle import rect
    p = fps.plan(n, tol=1e-13, box=box, host_only=True)
    J, po, qo = rect.rect_shifts(n, box, 1e-13)
    assert p.J == J
    pl, ql = p.shift_pairs()
    scale = max(abs(v) for v in rect.rect_enclosure(n, box))
    np.testing.assert_allclose(pl, po[::-1], rtol=1e-13, atol=1e-15 * scale)
    np.testing.assert_allclose(ql, qo[::-1], rtol=1e-13, atol=1e-15 * scale)
    assert np.all(np.diff(np.abs(pl)) >= 0)
    assert p.out_entries == (n + 2) ** 2


def test_rect_plan_tight_and_refined():
    from oracle import rect
    box = RECT_BOXES[1]
    n = 256
    lam, _ = square.atilde_eig(n)
    lo, hi = lam.min() * (1 + 1e-6), lam.max() * (1 - 1e-6)
    p = fps.plan(n, tol=1e-13, box=box, host_only=True, tight=True)
    J, po, qo = rect.rect_shifts(n, box, 1e-13, lam=(lo, hi))
    assert p.J == J < fps.plan(n, tol=1e-13, box=box, host_only=True).J
    pl, ql = p.shift_pairs()
    np.testing.assert_allclose(pl, po[::-1], rtol=1e-8)
    np.testing.assert_allclose(ql, qo[::-1], rtol=1e-8)
    r = fps.plan(n, tol=1e-13, box=box, precision="fp32_refined", host_only=True)
    assert r.rounds == 3 and r.f32_steps == sum(r.round_steps()[0])
    rp = r.shift_pairs()[0]
    assert np.all(np.diff(np.abs(rp)) >= 0)  # increasing |p_j|, as FP64 plans
    # a unit box is the square plan
    u = fps.plan(n, tol=1e-13, box=(-1.0, 1.0, -1.0, 1.0), host_only=True)
    s = fps.plan(n, tol=1e-13, host_only=True)
    assert u.J == s.J
    np.testing.assert_allclose(u.shift_pairs()[0], s.shifts(), rtol=0, atol=0)


def test_rect_and_dirichlet_argument_errors():
    L = fps.lib()
    h = ctypes.c_void_p()
    for box in [(1.0, 1.0, 0.0, 1.0), (0.0, 1.0, 2.0, -2.0), (0.0, float("inf"), 0.0, 1.0),
                (float("nan"), 1.0, 0.0, 1.0)]:
        b = (ctypes.c_double * 4)(*box)
        assert L.fps_plan_create_rect(ctypes.byref(h), 16, b, 1e-13, 0, 0, 1) == 1, box
    b = (ctypes.c_double * 4)(0.0, 1.0, 0.0, 2.0)
    assert L.fps_plan_create_rect(ctypes.byref(h), 16, None, 1e-13, 0, 0, 1) == 1
    assert L.fps_plan_create_rect(ctypes.byref(h), 16, b, 1e-13, 0, 0, 4 | 1) == 1  # cube flag
    assert L.fps_plan_create_rect(ctypes.byref(h), 0, b, 1e-13, 0, 0, 1) == 1
    assert L.fps_plan_create(ctypes.byref(h), 3, 16, 0, 1e-13, 0, 0, 8 | 1) == 2  # cube + lift
    p = fps.plan(16, box=(0.0, 1.0, 0.0, 2.0), host_only=True, dirichlet=True)
    assert L.fps_solve_dirichlet(p.handle, None, None, None, None, None) == 5  # host-only
    assert L.fps_solve_dirichlet(None, None, None, None, None, None) == 5


@pytest.mark.parametrize("n", [1, 2, 5, 64, 201])
def test_lift_map_matches_oracle(shim, n):
    # Ms[s][a][b] = C~_{2a+s} coefficient of T''_{2b+s} / sqrt((i+1)(i+2)):
    # against the oracle's extended-precision projection of each T_k''
    from oracle import rect
    m = [(n + 1) // 2, n // 2]
    mo = [(n + 3) // 2, (n + 2) // 2]
    M0 = np.zeros(m[0] * mo[0])
    M1 = np.zeros(max(m[1] * mo[1], 1))
    P = ctypes.POINTER(ctypes.c_double)
    shim.shim_lift_map(n, M0.ctypes.data_as(P), M1.ctypes.data_as(P))
    N = n + 2
    R = rect.cheb_to_ct_closed(n, n, dtype=np.longdouble)
    full = np.zeros((n, N))
    for k in range(N):
        e = np.zeros(N, dtype=np.longdouble)
        e[k] = 1
        d2 = rect.cheb_second_derivative(e)
        full[:, k] = (R @ d2[:n] if len(d2) >= n else R[:, :len(d2)] @ d2).astype(np.float64)
    i = np.arange(n)
    full /= np.sqrt((i + 1.0) * (i + 2.0))[:, None]
    for s, Ms in ((0, M0), (1, M1)):
        if m[s] == 0:
            continue
        got = Ms[: m[s] * mo[s]].reshape(m[s], mo[s])
        want = full[s::2, s::2]
        # the oracle side projects each T_k'' (coefficients up to ~k^3) in
        # extended precision, cancelling by up to ~1e6: 1e-12 relative
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=0)


@pytest.mark.parametrize("n", [2, 8, 20, 64])
def test_cylinder_mode_bands_match_oracle(n):
    # closed-form derivative matrices and powers of the C~ Jacobi matrix in
    # the library against the oracle's quadrature Galerkin matrices
    from oracle import cylinder
    for k in (0, 1, -1, 2, 3, 6, 17):
        P, Q = fps.cylinder_mode_bands(n, k)
        Po, Qo, _, _, wp, rp = cylinder.mode_operators(n, k)
        ri, wi = np.arange(rp, n, 2), np.arange(wp, n, 2)
        Pr, Qr = Po[np.ix_(ri, wi)], Qo[np.ix_(ri, wi)]
        m = n // 2
        Pd, Qd = np.zeros((m, m)), np.zeros((m, m))
        for a in range(m):
            for c in range(5):
                b = a + c - 2
                if 0 <= b < m:
                    Pd[a, b], Qd[a, b] = P[a, c], Q[a, c]
        assert np.abs(Pd - Pr).max() <= 1e-12 * np.abs(Pr).max(), (n, k)
        assert np.abs(Qd - Qr).max() <= 1e-12 * np.abs(Qr).max(), (n, k)


def test_cylinder_plan_queries_and_errors():
    p = fps.plan_cylinder(16, 8, host_only=True)
    assert p.J == 0
    assert p.out_entries == 8 * 2 * 20 * 18
    assert p.out_shape() == (8, 2, 20, 18) and p.in_shape() == (8, 2, 16, 16)
    L = fps.lib()
    h = ctypes.c_void_p()
    assert L.fps_plan_create_cylinder(ctypes.byref(h), 15, 8, 1) == 1  # odd n
    assert L.fps_plan_create_cylinder(ctypes.byref(h), 16, 7, 1) == 1  # odd n_theta
    assert L.fps_plan_create_cylinder(ctypes.byref(h), 16, 8, 2) == 1  # flags
    assert L.fps_plan_create_cylinder(ctypes.byref(h), 1024, 8, 1) == 2
    assert L.fps_solve_adjoint(p.handle, None, None, None, None) == 5  # host-only
