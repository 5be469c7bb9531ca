"""Benchmark: square Poisson solve (F_T -> U), n = 4096, FP64, on one MI355X.

One step = one full solve through the C ABI: Chebyshev -> C~ input map,
the 2J ADI half-sweeps of Algorithm 2, and the output map to the (n+2)^2
Chebyshev coefficients.  Inputs are resident in HBM before timing starts.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "dof/s, square Poisson n=4096 at rel err ≤1e-12; % of HBM roofline"
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6  # dense FP64 matrix peak of MI355X
# Calibrated HBM traffic of the sweep kernels per launch (rocprofv3
# FETCH_SIZE x1.9999 + WRITE_SIZE x1.0000, see profiles/sweep_square_n4096.md
# and profiles/sweep_square_n10000.md), valid only for the sweep source
# (sweep.hip) with this sha256 (the counters were taken on the same device
# code).
SWEEP_SOURCES = ("sweep.hip",)
SWEEP_TRAFFIC = {"sha256": "26523be850a96aee6cae29ca6125c86917afec02f83fb7294da6db3a9528f947",
                 4096: {"half_step_1": 277.6e6, "half_step_2": 413.0e6},
                 10000: {"half_step_1": 1764.2e6, "half_step_2": 2529.8e6}}


def sweep_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(os.path.join(ROOT, "paper_1710_11259_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def sweep_traffic(n):
    """Counter-measured HBM bytes per sweep launch at size n, mean of the two
    half-steps, or None when the sources changed since the counters were
    taken (or no counters exist for n)."""
    if sweep_sources_sha() != SWEEP_TRAFFIC["sha256"] or n not in SWEEP_TRAFFIC:
        return None
    t = SWEEP_TRAFFIC[n]
    return (t["half_step_1"] + t["half_step_2"]) / 2.0


def copy_rate(torch, dev, mib=1024, reps=5):
    """Achievable HBM rate of a plain copy kernel: GB/s (bytes read plus
    bytes written) of a device-to-device copy of `mib` MiB, far larger than
    the last-level cache."""
    nbytes = mib << 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def stream_rate(fps, torch, dev, mib=1024, reps=5):
    """Achievable HBM rate of the library's own streaming pass
    (fps.probe_stream: c = a + b, two reads and one write per element in
    16-byte accesses) on three arrays of `mib` MiB each, far larger than the
    last-level cache: GB/s of bytes read plus bytes written."""
    nel = (mib << 20) // 8
    a = torch.ones(nel, dtype=torch.float64, device=dev)
    b = torch.full((nel,), 2.0, dtype=torch.float64, device=dev)
    c = torch.empty_like(a)
    fps.probe_stream(a, b, c)
    torch.cuda.synchronize()
    ok = bool((c[:: max(1, nel // 4096)] == 3.0).all())
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fps.probe_stream(a, b, c)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b, c
    torch.cuda.empty_cache()
    return {"GBs": round(3.0 * nel * 8 / (ms * 1e-3) / 1e9, 1), "array_MiB": mib, "arrays": 3,
            "us_per_pass": round(ms * 1e3, 2), "result_ok": ok}


def host_info():
    """The host the oracle runs on: CPU model, logical CPUs this process may
    use, and the BLAS library numpy and scipy call with its thread count."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cpus = len(os.sched_getaffinity(0))
    except AttributeError:
        cpus = os.cpu_count()
    blas = []
    try:
        import threadpoolctl
        for d in threadpoolctl.threadpool_info():
            blas.append({k: d.get(k) for k in ("user_api", "internal_api", "version",
                                               "num_threads", "threading_layer", "architecture")})
    except Exception as exc:  # threadpoolctl missing or failing: say so
        blas.append({"error": repr(exc)})
    threads = max([d.get("num_threads") or 1 for d in blas if "num_threads" in d] or [1])
    return {"cpu_model": model, "cpus_available": cpus, "blas": blas, "blas_threads": threads}


def time_oracle(fn, reps=3):
    """One warm-up call, then `reps` timed calls: (median seconds, all times,
    the warm-up call's result)."""
    import statistics
    res = fn()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        times.append(time.perf_counter() - t0)
    return statistics.median(times), times, res


_CUBE_ORACLE = {}


def cube_oracle(F_host, n):
    """The oracle's cube solution for the benchmark's cube input (computed
    once per run and shared by the cube forms), with its timing: warm-up
    plus the median of three solves."""
    if n not in _CUBE_ORACLE:
        from oracle import cube
        med, times, Uo = time_oracle(lambda: cube.poisson_cube(F_host))
        _CUBE_ORACLE[n] = (Uo, med, times)
    return _CUBE_ORACLE[n]


def graph_timing(fps, torch, p, F, U_eager, steps):
    """The same solve captured into one HIP graph (fps.SolveGraph): ms per
    replay and whether the replay equals the eager result bit for bit.  The
    capture removes the host's per-launch cost, which shows where a solve
    issues many short launches."""
    g = fps.SolveGraph(p)
    g.F.copy_(F)
    g.replay()
    torch.cuda.synchronize()
    same = bool(torch.equal(g.U, U_eager))
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    del g
    torch.cuda.empty_cache()
    return ms, same


def calibration_copy(torch, dev, mib):
    """One device-to-device copy of a known size (HBM counter calibration)."""
    nbytes = mib << 20
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    print(f"# calibration copy {nbytes} bytes read + {nbytes} bytes written", file=sys.stderr)


def bench_batch(fps, workloads, torch, tol, reps=3, tight=True):
    """256 independent square solves (n_b = 32 U{1..32}, seed 1): one graph
    launch per batch (FP64 and FP32-refined) against a sequential loop of
    single FP64 solves, run eagerly and replayed from one HIP graph per
    solve."""
    import numpy as np
    ns, Fs = workloads.batched_problems()
    dof = float(sum(n * n for n in ns))
    res = {"problems": len(ns), "dof": dof,
           "enclosure": "computed spectrum" if tight else "Lemma B.1"}
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(k):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / k

    # sequential single FP64 solves (the same inputs, one plan per size)
    plans = {n: fps.plan(n, tol=tol, tight=tight) for n in sorted(set(ns))}
    ws = torch.empty(max(p.workspace_bytes for p in plans.values()), dtype=torch.uint8,
                     device="cuda")
    Fd = [torch.from_numpy(F).cuda() for F in Fs]
    Us = [torch.empty(plans[n].out_shape(), dtype=torch.float64, device="cuda") for n in ns]

    def seq():
        for n, F, U in zip(ns, Fd, Us):
            fps.solve(plans[n], F, out=U, ws=ws)
    t_seq = timed(seq, 1)
    res["sequential_fp64_ms"] = t_seq
    # the same solves, each captured into its own HIP graph (no host launch
    # cost inside a solve): the device-side baseline of the batched launches
    graphs = []
    for n, F in zip(ns, Fd):
        g1 = fps.SolveGraph(plans[n])
        g1.F.copy_(F)
        graphs.append(g1)

    def seq_graphs():
        for g1 in graphs:
            g1.replay()
    t_seq_graph = timed(seq_graphs, reps)
    res["sequential_fp64_graph_equals_eager"] = all(
        bool(torch.equal(g1.U, U)) for g1, U in zip(graphs, Us))
    res["sequential_fp64_graph_ms"] = t_seq_graph
    del graphs
    for prec in ("fp64", "fp32_refined"):
        b = fps.batch(ns, tol=tol, precision=prec, tight=tight)
        g = fps.BatchGraph(b)
        g.F.copy_(b.pack(Fs))
        t = timed(g.replay, reps)
        r = {"ms_per_batch": t, "dof_per_s": dof / (t * 1e-3), "speedup_vs_sequential_fp64":
             t_seq / t, "speedup_vs_sequential_fp64_graph": t_seq_graph / t, "max_J": b.max_J,
             "launch": "one HIP graph"}
        got = b.unpack(g.U)
        worst = 0.0
        for U, Ub in zip(Us, got):
            d = float(torch.linalg.norm(Ub - U) / torch.linalg.norm(U))
            worst = max(worst, d)
        r["max_rel_diff_vs_sequential_fp64"] = worst
        res[prec] = r
        del g, b
    del ws
    torch.cuda.empty_cache()
    return res


def bench_cube(fps, workloads, torch, tol, n=256, steps=2, check=True, tight=True):
    """Cube n^3 solve (two-level nested ADI, FP64): time per solve and the
    fiber sweeps' achieved bandwidth.  Algorithmic bytes per dof: z sweep 24
    (read zR and B, write), inner half-step 1 16, half-step 2 24; for parity
    blocks of at most 128 the inner ADI of an outer step is one LDS-resident
    launch (HBM: R read into LDS, into registers and for the outer update,
    B read, the next zR written: 32 B per dof)."""
    import numpy as np
    F_host = workloads.cube_rhs(n)
    F = torch.from_numpy(F_host).cuda()
    p = fps.plan(n, tol=tol, dim=3, tight=tight)
    counts = p.inner_counts()
    ws = fps.workspace(p, "cuda")
    U = torch.empty(p.out_shape(), dtype=torch.float64, device="cuda")
    fps.solve(p, F, out=U, ws=ws)
    torch.cuda.synchronize()
    per_solve = sum(1 + 2 * c for c in counts)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fps.solve(p, F, out=U, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # one more solve with an event pair around every sweep launch
    p.set_sweep_timing(per_solve)
    e0.record()
    fps.solve(p, F, out=U, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    ms_instr = e0.elapsed_time(e1)
    t = p.sweep_time()
    p.set_sweep_timing(0)
    dof = float(n) ** 3
    # parity blocks of at most 128 run every outer step's inner ADI as one
    # LDS-resident launch: the timed launches alternate z sweep, inner ADI
    lds = len(t) == 2 * len(counts)
    kinds = []
    for c in counts:
        kinds.append("z")
        kinds.extend(["inner"] if lds else ["hs1", "hs2"] * c)
    bpd = {"z": 24.0, "hs1": 16.0, "hs2": 24.0, "inner": 24.0}
    sweep_kinds = ("z",) if lds else ("z", "hs1", "hs2")
    tot_b = sum(bpd[k] * dof for k in kinds[:len(t)] if k in sweep_kinds)
    tot_t = sum(x for x, k in zip(t, kinds) if k in sweep_kinds) * 1e-3
    res = {"n": n, "dof": dof, "ms_per_solve": ms, "dof_per_s": dof / (ms * 1e-3),
           "enclosure": "computed spectrum" if tight else "Lemma B.1",
           "J_outer": p.J, "inner_steps": sum(counts),
           "sweeps_per_solve": len(counts) if lds else per_solve,
           "sweep_achieved_GBs": round(tot_b / tot_t / 1e9, 1),
           "sweep_frac_of_8TBs": round(tot_b / tot_t / 8e12, 4),
           "sweep_share_of_solve": round(sum(t) / ms_instr, 4)}
    if lds:
        ti = [x for x, k in zip(t, kinds) if k == "inner"]
        # the streamed inner passes it replaces: 40 B per dof and inner step
        res["inner_adi"] = {
            "form": "one launch per outer step, every slice block resident in LDS",
            "launches": len(ti), "ms_total": round(sum(ti), 3),
            "share_of_solve": round(sum(ti) / ms_instr, 4),
            "hbm_bytes_per_launch": 4 * 8 * dof,
            "sweep_model_bytes": 40.0 * dof * sum(counts),
            "sweep_model_equiv_GBs": round(40.0 * dof * sum(counts) / (sum(ti) * 1e-3) / 1e9, 1)}
    for k in ("z", "hs1", "hs2"):
        tk = [x for x, kk in zip(t, kinds) if kk == k]
        if tk:
            avg = sum(tk) / len(tk) * 1e-3
            res[f"avg_us_{k}"] = round(avg * 1e6, 2)
            res[f"GBs_{k}"] = round(bpd[k] * dof / avg / 1e9, 1)
    if check:
        Uo = cube_oracle(F_host, n)[0]
        Ug = U.cpu().numpy()
        res["rel_frobenius_err_vs_oracle"] = float(np.linalg.norm(Ug - Uo) / np.linalg.norm(Uo))
        res["max_abs_ratio_vs_oracle"] = float(np.abs(Ug - Uo).max() / np.abs(Uo).max())
    del ws
    torch.cuda.empty_cache()
    return res


def bench_cube_zeig(fps, workloads, torch, tol, n=256, steps=3, check=True, tight=True):
    """Cube n^3 solve through the z-eigenbasis (one ADI per z-slice, FP64):
    time per solve, and the ADI's own figures: for n <= 256 the one launch
    that keeps every slice block in LDS (its time, its HBM bytes, and the
    streamed sweeps' bytes per the same time), else the batched slice
    sweeps' achieved bandwidth.  Sweep-model bytes per slice and step: x
    solve 16 n^2, y solve 24 n^2."""
    import numpy as np
    F_host = workloads.cube_rhs(n)
    F = torch.from_numpy(F_host).cuda()
    p = fps.plan(n, tol=tol, dim=3, tight=tight, zeig=True)
    counts = p.slice_counts()
    ws = fps.workspace(p, "cuda")
    U = torch.empty(p.out_shape(), dtype=torch.float64, device="cuda")
    fps.solve(p, F, out=U, ws=ws)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fps.solve(p, F, out=U, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # launch sequence of one solve: (slices, bytes per slice)
    seq = []
    Jmax = max(counts) if counts else 0
    for j in range(Jmax):
        k1 = sum(1 for c in counts if c > j)
        seq.append((k1, 16.0))
        seq.append((k1, 24.0))
    p.set_sweep_timing(len(seq))
    e0.record()
    fps.solve(p, F, out=U, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    ms_instr = e0.elapsed_time(e1)
    t = p.sweep_time()
    p.set_sweep_timing(0)
    ms_g, same_g = graph_timing(fps, torch, p, F, U, steps)
    dof = float(n) ** 3
    res = {"n": n, "dof": dof, "ms_per_solve": ms, "dof_per_s": dof / (ms * 1e-3),
           "enclosure": "computed spectrum" if tight else "Lemma B.1",
           "method": "eigenbasis of A~ along z (MFMA transforms), one ADI per z-slice",
           "slice_steps": sum(counts), "max_slice_J": Jmax,
           "hip_graph": {"ms_per_solve": ms_g, "dof_per_s": dof / (ms_g * 1e-3),
                         "equals_eager": same_g}}
    sweep_model = sum(k * b * n * n for k, b in seq)  # 40 B per dof and slice step
    if len(t) == 1:
        # every slice's ADI in one launch, each parity block LDS-resident: HBM
        # sees G^ read and Y^ written once (npad^3 each); the sweep model's
        # bytes over the kernel's time give the rate the streamed form would
        # need for the same time
        npad = ((n + 1) // 2 + 63) // 64 * 64 + (n // 2 + 63) // 64 * 64
        hbm_b = 2 * 8.0 * npad ** 3
        res["adi"] = {"form": "one launch, every slice block resident in LDS",
                      "kernel_ms": round(t[0], 4), "share_of_solve": round(t[0] / ms_instr, 4),
                      "hbm_bytes": hbm_b, "hbm_GBs": round(hbm_b / (t[0] * 1e-3) / 1e9, 1),
                      "sweep_model_bytes": sweep_model,
                      "sweep_model_equiv_GBs": round(sweep_model / (t[0] * 1e-3) / 1e9, 1)}
    else:
        tot_b = sum(k * b * n * n for k, b in seq[:len(t)])
        tot_t = sum(t) * 1e-3
        res["adi"] = {"form": "batched slice sweeps", "sweep_launches": len(seq),
                      "sweep_achieved_GBs": round(tot_b / tot_t / 1e9, 1),
                      "sweep_frac_of_8TBs": round(tot_b / tot_t / 8e12, 4),
                      "sweep_share_of_solve": round(sum(t) / ms_instr, 4)}
    # FP32 storage + FP64 refinement (rounds of the K-form slice correction)
    pr = fps.plan(n, tol=tol, dim=3, tight=tight, zeig=True, precision="fp32_refined")
    wsr = fps.workspace(pr, "cuda")
    Ur = torch.empty(pr.out_shape(), dtype=torch.float64, device="cuda")
    fps.solve(pr, F, out=Ur, ws=wsr)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        fps.solve(pr, F, out=Ur, ws=wsr)
    e1.record()
    torch.cuda.synchronize()
    ms_r = e0.elapsed_time(e1) / steps
    rsteps, rtols = pr.round_steps()
    res["fp32_refined"] = {"ms_per_solve": ms_r, "dof_per_s": dof / (ms_r * 1e-3),
                           "speedup_vs_fp64": ms / ms_r, "rounds": pr.rounds,
                           "round_max_slice_J": rsteps, "round_tols": rtols,
                           "round0_slice_steps": sum(pr.slice_counts())}
    if check:
        Uo, med, times = cube_oracle(F_host, n)
        Ug = U.cpu().numpy()
        res["rel_frobenius_err_vs_oracle"] = float(np.linalg.norm(Ug - Uo) / np.linalg.norm(Uo))
        res["max_abs_ratio_vs_oracle"] = float(np.abs(Ug - Uo).max() / np.abs(Uo).max())
        hi = host_info()
        res["cpu_baseline"] = {
            "value": dof / med, "unit": "dof/s", "cores": hi["blas_threads"], "kind": "oracle",
            "sample": f"full n={n} cube solves by the oracle (Kronecker eigenbasis: three "
                      f"mode products each way, numpy/OpenBLAS FP64), one warm-up then the "
                      f"median of {len(times)}: " + ", ".join(f"{t:.2f}" for t in times) + " s",
            "host": hi}
        Urh = Ur.cpu().numpy()
        res["fp32_refined"]["rel_frobenius_err_vs_oracle"] = float(
            np.linalg.norm(Urh - Uo) / np.linalg.norm(Uo))
        res["fp32_refined"]["max_abs_ratio_vs_oracle"] = float(
            np.abs(Urh - Uo).max() / np.abs(Uo).max())
    del ws, wsr
    torch.cuda.empty_cache()
    return res


def bench_rect_dirichlet(fps, workloads, torch, tol, n=4096, box=(0.0, 2.5, -1.0, 0.25), steps=5,
                         check=True, tight=True):
    """Rectangle [0, 2.5] x [-1, 0.25] with nonzero Dirichlet data (four random
    traces, corners matched), FP64: time per solve with the device-side lift,
    and the same plan's zero-data solve for the lift's overhead."""
    import numpy as np
    F_host, bc_host = workloads.rect_dirichlet_case(n, seed=5)
    F = torch.from_numpy(F_host).cuda()
    bc = torch.from_numpy(bc_host).cuda()
    p = fps.plan(n, tol=tol, box=box, tight=tight, dirichlet=True)
    ws = fps.workspace(p, "cuda")
    U = torch.empty(p.out_shape(), dtype=torch.float64, device="cuda")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms_d = timed(lambda: fps.solve_dirichlet(p, F, bc, out=U, ws=ws))
    Ud = U.cpu().numpy()
    ms_0 = timed(lambda: fps.solve(p, F, out=U, ws=ws))
    res = {"n": n, "box": list(box), "dof": float(n) ** 2, "J": p.J,
           "ms_per_solve": ms_d, "dof_per_s": n * n / (ms_d * 1e-3),
           "ms_zero_data_same_plan": ms_0, "lift_overhead_ms": ms_d - ms_0,
           "enclosure": "computed spectrum" if tight else "Lemma B.1",
           "shifts": "general (p_j != -q_j): two tables per step"}
    if check:
        from oracle import rect
        Uo = rect.poisson_rect_dirichlet(F_host, bc_host, box)
        res["rel_frobenius_err_vs_oracle"] = float(np.linalg.norm(Ud - Uo) / np.linalg.norm(Uo))
        tr = rect.boundary_traces(Ud)
        res["max_trace_err"] = float(max(np.abs(a - b).max() for a, b in zip(tr, bc_host)))
    del ws
    torch.cuda.empty_cache()
    return res


def bench_cylinder(fps, workloads, torch, n=256, n_theta=256, steps=5, check=True):
    """Cylinder (Sec. 4.1), n Chebyshev coefficients in r and z, n_theta
    Fourier modes, FP64: time per solve (the per-mode systems solved
    exactly in the z-eigenbasis), plan time, and the oracle's per-mode
    solution on a sample of modes covering the three cases."""
    import time as _t
    import numpy as np
    F_host = workloads.cylinder_rhs(n, n_theta, seed=9)
    F = torch.from_numpy(np.ascontiguousarray(np.stack([F_host.real, F_host.imag], axis=1))).cuda()
    t0 = _t.perf_counter()
    p = fps.plan_cylinder(n, n_theta)
    t_plan = _t.perf_counter() - t0
    ws = fps.workspace(p, "cuda")
    U = torch.empty(p.out_shape(), dtype=torch.float64, device="cuda")
    fps.solve(p, F, out=U, ws=ws)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fps.solve(p, F, out=U, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    ms_g, same_g = graph_timing(fps, torch, p, F, U, steps)
    dof = float(n) * n * n_theta
    # Whole-solve rooflines.  MFMA: the four maps, 6 n_theta n^3 flops (z in and
    # out 2 n_theta n^3 each, r in and out n_theta n^3 each, parity blocks).
    # HBM: every stage reads its operands and writes its result once: the
    # permutation (F, X), the z and r input maps (2 X each), the banded solves
    # (factor table + 2 X), the z output map (X + X_out), the r output map
    # (X_out + U) and the fill of U; X = 2 n_theta npad^2 doubles, X_out with
    # the padded z output width.
    m = n // 2
    mp = (m + 63) // 64 * 64
    npad = 2 * mp
    mobar = 2 * ((m + 1 + 63) // 64 * 64)
    X = 2.0 * n_theta * npad * npad * 8
    Xo = X * mobar / npad
    Fb = 2.0 * n_theta * n * n * 8
    Ub = 2.0 * n_theta * (n + 4) * (n + 2) * 8
    fac = (n_theta // 2 + 1) * 8.0 * mp * npad * 8
    hbm = (Fb + X) + 2 * X + 2 * X + (fac + 2 * X) + (X + Xo) + (Xo + Ub) + Ub
    flops = 6.0 * n_theta * float(n) ** 3
    res = {"n": n, "n_theta": n_theta, "dof": dof, "ms_per_solve": ms,
           "dof_per_s": dof / (ms * 1e-3), "plan_s": round(t_plan, 2),
           "hip_graph": {"ms_per_solve": ms_g, "dof_per_s": dof / (ms_g * 1e-3),
                         "equals_eager": same_g},
           "method": "z-eigenbasis of A~, host-factored banded r-solves per (mode, z column), "
                     "MFMA GEMM maps",
           "roofline_whole_solve": {
               "hbm_bytes_algorithmic": hbm, "hbm_GBs": round(hbm / (ms * 1e-3) / 1e9, 1),
               "hbm_frac": round(hbm / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               "mfma_flops": flops, "TFLOPs": round(flops / (ms * 1e-3) / 1e12, 2),
               "fp64_mfma_frac": round(flops / (ms * 1e-3) / 1e12 / FP64_MFMA_PEAK_TFLOPS, 4)}}
    if check:
        from oracle import cylinder
        Ug = U.cpu().numpy()
        worst = 0.0
        for k in (0, 1, -1, 2, -3, 17, n_theta // 4, -(n_theta // 2), n_theta // 2 - 1):
            idx = k + n_theta // 2
            Uo = (cylinder.solve_mode(np.ascontiguousarray(F_host[idx].real), k)
                  + 1j * cylinder.solve_mode(np.ascontiguousarray(F_host[idx].imag), k))
            Uk = Ug[idx, 0] + 1j * Ug[idx, 1]
            worst = max(worst, float(np.linalg.norm(Uk - Uo) / np.linalg.norm(Uo)))
        res["rel_err_vs_oracle_sampled_modes"] = worst
    del ws
    torch.cuda.empty_cache()
    return res


def bench_square_large(fps, workloads, torch, tol, n=10000, steps=3, check=True, tight=True):
    """The square at n = 10^4 (10^8 dof, the size of the paper's own timing
    example): time per FP64 solve and the error against the oracle's exact
    discrete solution."""
    import numpy as np
    F_host = workloads.square_rhs(n, seed=0)
    F = torch.from_numpy(F_host).cuda()
    p = fps.plan(n, tol=tol, tight=tight)
    ws = fps.workspace(p, "cuda")
    U = torch.empty(p.out_shape(), dtype=torch.float64, device="cuda")
    fps.solve(p, F, out=U, ws=ws)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fps.solve(p, F, out=U, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # one more solve with an event pair around every sweep launch: at this
    # size no array fits the last-level cache, so the rate is HBM's alone
    p.set_sweep_timing(2 * p.J)
    fps.solve(p, F, out=U, ws=ws)
    torch.cuda.synchronize()
    t = p.sweep_time()
    p.set_sweep_timing(0)
    dof = float(n) * n
    t1 = sum(t[0::2]) / max(len(t[0::2]), 1) * 1e-3
    t2 = sum(t[1::2]) / max(len(t[1::2]), 1) * 1e-3
    b1, b2 = 16.0 * dof, 24.0 * dof
    res = {"n": n, "dof": dof, "J": p.J, "ms_per_solve": ms,
           "dof_per_s": dof / (ms * 1e-3),
           "paper_context": "10^8 dof in under two minutes on a 2017 laptop (MATLAB, one core)",
           "sweep": {"n": n, "bytes_per_launch": {"half_step_1": b1, "half_step_2": b2},
                     "avg_launch_us": {"half_step_1": round(t1 * 1e6, 2),
                                       "half_step_2": round(t2 * 1e6, 2)},
                     "achieved_GBs": round((b1 + b2) / (t1 + t2) / 1e9, 1),
                     "frac": round((b1 + b2) / (t1 + t2) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": sweep_traffic(n),
                     "launches_timed": len(t)}}
    if check:
        from oracle import square
        Uo = square.poisson_square(F_host)
        Ug = U.cpu().numpy()
        res["rel_frobenius_err_vs_oracle"] = float(np.linalg.norm(Ug - Uo) / np.linalg.norm(Uo))
        res["max_abs_ratio_vs_oracle"] = float(np.abs(Ug - Uo).max() / np.abs(Uo).max())
    del ws, U, F
    torch.cuda.empty_cache()
    return res


def bench_adjoint(fps, workloads, torch, tol, n=2048, batch=16, steps=3, check=True, tight=True):
    """Differentiation form: one forward and one backward pass of the autograd
    solve over a batch of 16 right-hand sides at n = 2048, for the quadratic
    loss ||U(F) - U*||^2 (U* the solution for a fixed target right-hand side).
    The backward pass is the adjoint solve (the same ADI sweeps between the
    transposed coefficient maps); nothing is stored from the forward pass."""
    import numpy as np
    F_host, Fstar, _ = workloads.adjoint_case(n, batch, n_dirs=1)
    p = fps.plan(n, tol=tol, tight=tight)
    Ustar = fps.solve(p, torch.from_numpy(Fstar).cuda())
    F = torch.from_numpy(F_host).cuda().requires_grad_(True)

    def step():
        F.grad = None
        U = fps.solve_fn(F, p)
        loss = ((U - Ustar) ** 2).sum()
        loss.backward()
        return U

    step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        U = step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    dof = float(batch) * n * n
    # algorithmic sweep bytes: 40 B per dof per ADI iteration, forward and backward
    sweep_bytes = 2.0 * batch * p.J * 40.0 * n * n
    res = {"n": n, "batch": batch, "J": p.J, "ms_per_fwd_bwd": ms,
           "dof_per_s": dof / (ms * 1e-3),
           "sweep_bytes_algorithmic": sweep_bytes,
           "sweep_bytes_rate_GBs": round(sweep_bytes / (ms * 1e-3) / 1e9, 1),
           "method": "autograd Function over one fps_batch: forward fps_batch_solve, backward "
                     "fps_batch_solve_adjoint (the sweeps of all problems in one launch per "
                     "half-step)"}
    if check:
        from oracle import adjoint
        Ub = (2.0 * (U[0] - Ustar)).detach().cpu().numpy()
        ref = adjoint.vjp_square(Ub, np.asarray(p.shifts(), dtype=float))
        got = F.grad[0].cpu().numpy()
        res["rel_err_vs_oracle_vjp_problem0"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    del F, U, Ustar
    torch.cuda.empty_cache()
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--tol", type=float, default=1e-13)
    ap.add_argument("--enclosure", choices=["tight", "lemma"], default="tight",
                    help="shift intervals: computed spectrum (default) or the Lemma B.1 enclosure")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the FP32-refined, batched, cube, rectangle and cylinder timings")
    ap.add_argument("--only", choices=["fp32_refined", "batched", "cube", "cube_zeig",
                                       "rect_dirichlet", "cylinder", "adjoint", "square_n10000"],
                    help="run only this form and print its figures (profiling)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one device-to-device copy of this size first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; sharding across GPUs is not "
                                   "implemented"}))
        return 2

    import numpy as np
    import torch

    import paper_1710_11259_amd as fps
    import workloads

    n = args.n
    dev = torch.device("cuda:0")
    if args.only in ("batched", "cube", "cube_zeig", "rect_dirichlet", "cylinder", "adjoint",
                     "square_n10000"):
        if args.copy_calib_mib:
            calibration_copy(torch, dev, args.copy_calib_mib)
        tight = args.enclosure == "tight"
        if args.only == "batched":
            res = bench_batch(fps, workloads, torch, args.tol, tight=tight)
        elif args.only == "cube":
            res = bench_cube(fps, workloads, torch, args.tol, steps=max(1, args.steps),
                             check=not args.no_check, tight=tight)
        elif args.only == "cylinder":
            res = bench_cylinder(fps, workloads, torch, steps=max(1, args.steps),
                                 check=not args.no_check)
        elif args.only == "rect_dirichlet":
            res = bench_rect_dirichlet(fps, workloads, torch, args.tol, n=n,
                                       steps=max(1, args.steps), check=not args.no_check,
                                       tight=tight)
        elif args.only == "adjoint":
            res = bench_adjoint(fps, workloads, torch, args.tol, steps=max(1, args.steps),
                                check=not args.no_check, tight=tight)
        elif args.only == "square_n10000":
            res = bench_square_large(fps, workloads, torch, args.tol, steps=max(1, args.steps),
                                     check=not args.no_check, tight=tight)
        else:
            res = bench_cube_zeig(fps, workloads, torch, args.tol, steps=max(1, args.steps),
                                  check=not args.no_check, tight=tight)
        print(json.dumps({"form": args.only, **res}), flush=True)
        return 0
    F_host = workloads.square_rhs(n, seed=0)
    F = torch.from_numpy(F_host).to(dev)
    tight = args.enclosure == "tight"
    plan = fps.plan(n, tol=args.tol, tight=tight)
    ws = fps.workspace(plan, dev)
    U = torch.empty(plan.out_shape(), dtype=torch.float64, device=dev)
    print(f"# plan n={n} J={plan.J} ws={plan.workspace_bytes / 2**20:.1f} MiB", file=sys.stderr,
          flush=True)

    if args.copy_calib_mib:
        calibration_copy(torch, dev, args.copy_calib_mib)

    for _ in range(args.warmup):
        fps.solve(plan, F, out=U, ws=ws)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    # Timed region: exactly `steps` solves, no instrumentation.
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        fps.solve(plan, F, out=U, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    # Roofline pass: the same solves again, every half-sweep launch carrying
    # a HIP event pair that records the dispatch's own start and end on the
    # solve's stream.
    plan.set_sweep_timing(2 * plan.J * args.steps)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        fps.solve(plan, F, out=U, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    instr_ms = e0.elapsed_time(e1)
    sweep_list = plan.sweep_time()
    plan.set_sweep_timing(0)
    ms_per_step = total_ms / args.steps
    dof = float(n) * float(n)
    value = dof / (ms_per_step * 1e-3)

    # Dominant kernel: the ADI half-sweep (k_sweep), two variants.
    # Algorithmic bytes per launch (24 B per dof would be read input + read G
    # + write output; here G is read by half-step 2 only):
    #   half-step 1: read input, write output           -> 16 B per dof
    #   half-step 2: read input, read G, write output   -> 24 B per dof
    J = plan.J
    hs1 = sweep_list[0::2]
    hs2 = sweep_list[1::2]
    t1 = sum(hs1) / max(len(hs1), 1) * 1e-3
    t2 = sum(hs2) / max(len(hs2), 1) * 1e-3
    b1, b2 = 16.0 * dof, 24.0 * dof
    achieved = (b1 + b2) / (t1 + t2) / 1e9
    traffic = sweep_traffic(n)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_note": "calibrated HBM bytes per launch, mean of the two half-steps "
                                f"(algorithmic mean {(b1 + b2) / 2:.4g})" if traffic else
                                "null: sweep sources changed since the counters were taken",
                "kernel": "ADI half-sweeps (k_sweep_rows: half-step 1, k_sweep: half-step 2), "
                          "byte-weighted",
                "bytes_per_launch": {"half_step_1": b1, "half_step_2": b2},
                "avg_launch_us": {"half_step_1": round(t1 * 1e6, 2),
                                  "half_step_2": round(t2 * 1e6, 2)},
                "achieved_GBs": {"half_step_1": round(b1 / t1 / 1e9, 1),
                                 "half_step_2": round(b2 / t2 / 1e9, 1)},
                "launches_timed": len(sweep_list),
                "timing": "HIP events recording each sweep dispatch's start and end "
                          "(hipExtLaunchKernelGGL), separate pass of the same solves with "
                          "every launch on one stream (the timed solves run the two "
                          "row-parity blocks on two streams, half the chains per launch) "
                          f"({instr_ms / args.steps:.2f} ms per solve with the events)",
                "sweep_share_of_step": round(sum(sweep_list) / instr_ms, 4)}
    # Beside the sweep roofline: the rate a plain copy kernel achieves, and the
    # whole solve's algorithmic bytes (sweeps 40 B per dof per ADI iteration;
    # the map stages each read their input and write their output once:
    # permutation, two GEMM stages and transpose on the input side, finalize,
    # fill of U and two GEMM stages on the output side, 136 B per dof).
    copy_gbs = copy_rate(torch, dev)
    ceiling = stream_rate(fps, torch, dev)
    solve_bytes = (40.0 * J + 136.0) * dof
    roofline["copy_kernel_GBs"] = round(copy_gbs, 1)
    roofline["frac_of_copy_kernel"] = round(achieved / copy_gbs, 4)
    roofline["stream_kernel"] = ceiling
    roofline["frac_of_stream_kernel"] = round(achieved / ceiling["GBs"], 4)
    roofline["whole_solve"] = {
        "bytes_algorithmic": solve_bytes,
        "achieved_GBs": round(solve_bytes / (ms_per_step * 1e-3) / 1e9, 1),
        "frac": round(solve_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    out = {"metric": METRIC, "value": value, "unit": "dof/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"square [-1,1]^2 Poisson, zero Dirichlet, n={n} "
                                  f"({n}x{n} Chebyshev coefficients of f, "
                                  f"N(0,1)(1+j)^-2(1+k)^-2, seed 0), FP64, tol {args.tol:g}, "
                                  f"J={J} (shift intervals: "
                                  f"{'computed spectrum of A~' if tight else 'Lemma B.1 enclosure'}), "
                                  "one right-hand side",
                      "n": n, "J": J, "tol": args.tol,
                      "enclosure": "computed spectrum" if tight else "Lemma B.1"},
           "roofline": roofline}

    # Precision form: FP32 storage with FP64 refinement, same workload and tol.
    forms = {}
    if not args.no_forms or args.only == "fp32_refined":
        po = fps.plan(n, tol=args.tol, tight=not tight)
        wso = fps.workspace(po, dev)
        Uo_ = torch.empty(po.out_shape(), dtype=torch.float64, device=dev)
        fps.solve(po, F, out=Uo_, ws=wso)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            fps.solve(po, F, out=Uo_, ws=wso)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_o = e0.elapsed_time(e1) / args.steps
        forms["lemma_enclosure" if tight else "computed_spectrum"] = {
            "ms_per_step": ms_o, "dof_per_s": dof / (ms_o * 1e-3), "J": po.J}
        del wso, Uo_
        pr = fps.plan(n, tol=args.tol, precision="fp32_refined", tight=tight)
        wsr = fps.workspace(pr, dev)
        Ur = torch.empty(pr.out_shape(), dtype=torch.float64, device=dev)
        fps.solve(pr, F, out=Ur, ws=wsr)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            fps.solve(pr, F, out=Ur, ws=wsr)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_r = e0.elapsed_time(e1) / args.steps
        rsteps, rtols = pr.round_steps()
        forms["fp32_refined"] = {"ms_per_step": ms_r, "dof_per_s": dof / (ms_r * 1e-3),
                                 "speedup_vs_fp64": ms_per_step / ms_r,
                                 "rounds": pr.rounds, "round_steps": rsteps, "round_tols": rtols,
                                 "f32_steps": pr.f32_steps,
                                 "fp64_J": J,
                                 "sweep_bytes_per_dof": {
                                     "fp32_refined": 20 * pr.f32_steps
                                     + 40 * (sum(rsteps) - pr.f32_steps),
                                     "fp64": 40 * J}}
        del wsr
        if args.only is None:
            forms["batched"] = bench_batch(fps, workloads, torch, args.tol, tight=tight)
            forms["cube"] = bench_cube(fps, workloads, torch, args.tol, check=not args.no_check,
                                       tight=tight)
            forms["cube_zeig"] = bench_cube_zeig(fps, workloads, torch, args.tol,
                                                 check=not args.no_check, tight=tight)
            forms["rect_dirichlet"] = bench_rect_dirichlet(fps, workloads, torch, args.tol, n=n,
                                                           check=not args.no_check, tight=tight)
            forms["cylinder"] = bench_cylinder(fps, workloads, torch, check=not args.no_check)
            forms["adjoint"] = bench_adjoint(fps, workloads, torch, args.tol,
                                             check=not args.no_check, tight=tight)
            forms["square_n10000"] = bench_square_large(fps, workloads, torch, args.tol,
                                                        check=not args.no_check, tight=tight)
            sw = dict(forms["square_n10000"]["sweep"])
            sw["frac_of_stream_kernel"] = round(sw["achieved_GBs"] / ceiling["GBs"], 4)
            roofline["sweep_n10000"] = sw
    if forms:
        out["forms"] = forms

    Ug = U.cpu().numpy()
    if not args.no_cpu_baseline or not args.no_check:
        from oracle import square

        def oracle_solve():
            # the oracle's square solve (poisson_square), keeping its native X
            Xo_ = square.solve_native(square.rhs_ct(F_host))
            return Xo_, square.to_chebyshev(Xo_)

        if args.no_cpu_baseline:
            Xo, Uo = oracle_solve()
        else:
            t_cpu, t_all, (Xo, Uo) = time_oracle(oracle_solve)
        err = float(np.linalg.norm(Ug - Uo) / np.linalg.norm(Uo))
        # the same comparison on X (a native-output plan, outside the timing)
        pn = fps.plan(n, tol=args.tol, out="native", tight=tight)
        Xg = fps.solve(pn, F).cpu().numpy()
        del pn
        out["accuracy"] = {"rel_frobenius_err_vs_oracle": err,
                           "max_abs_ratio_vs_oracle": float(np.abs(Ug - Uo).max() / np.abs(Uo).max()),
                           "native_X": {"rel_frobenius": float(np.linalg.norm(Xg - Xo)
                                                               / np.linalg.norm(Xo)),
                                        "max_abs_ratio": float(np.abs(Xg - Xo).max()
                                                               / np.abs(Xo).max())},
                           "bound": 1e-12, "ok": bool(err <= 1e-12)}
        if "fp32_refined" in forms:
            er = float(np.linalg.norm(Ur.cpu().numpy() - Uo) / np.linalg.norm(Uo))
            forms["fp32_refined"]["rel_frobenius_err_vs_oracle"] = er
        if not args.no_cpu_baseline:
            hi = host_info()
            out["cpu_baseline"] = {
                "value": dof / t_cpu, "unit": "dof/s", "cores": hi["blas_threads"],
                "kind": "oracle",
                "sample": f"full n={n} solves by the FP64 eigen-decomposition oracle "
                          f"(numpy/scipy/OpenBLAS), one warm-up then the median of "
                          f"{len(t_all)}: " + ", ".join(f"{t:.2f}" for t in t_all) + " s",
                "host": hi}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
