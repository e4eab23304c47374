#!/usr/bin/env python3
"""Benchmark of the flexible shifted-Krylov solver on one MI355X.

Workload (the configuration the headline metric is quoted on): 2-D
finite-volume groundwater operator on a 512 x 512 grid (262,144 unknowns),
ln K ~ N(-11.5, 1) smoothed by a 5 x 5 box, Ss = 1e-5, h = 1; 200 shifts
sigma_j = i 2 pi / T_j with periods log-spaced 5..5000 s; one point source at
the centre; preconditioner shifts cycling over i*omega_{20,100,180}; inner
COCG tolerance 1e-6; restart 50; every shift to FP64 true relative residual
<= 1e-6 (refinement included).  A step is one complete solve of all 200
shifts with inputs resident on the device.

Prints one JSON line.  The value is shifted solves per second of the mixed
(complex64 bulk, FP64 least squares / residuals / refinement) path; the plain
FP64 path is timed the same way and reported beside it.  Unless --no-extra,
the line also carries the batched workloads (256x256 with 64 forward+adjoint
right-hand sides, 128^3 with 8), mixed and FP64 with all right-hand sides in
lockstep and, for 256x256, FP64 one right-hand side at a time.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "shifted solves/s at rel-res 1e-6 (mixed batched vs plain FP64); p50/p99 ms"
HBM_PEAK_GBS = 8000.0
BLOCK_M = 30   # block steps of the shared block basis (the batched workloads need 17-20)


def kernel_source_digest():
    h = hashlib.sha256()
    for f in ("kernels.hpp", "mg.hpp", "ops.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_1212_3660_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = int(math.floor(k)), int(math.ceil(k))
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def time_path(P, torch, gp, w, precision, steps, warmup, profile=False, precond=None, relax=0.0, variant=None):
    prm, keep = P.make_params(w.tau_seq, m_restart=w.m_restart, max_restarts=20, max_refine=4, tol=w.tol,
                              eps_inner=w.eps_inner, precision=precision,
                              inner_precond=P.SHK_PRECOND_MULTIGRID if precond is None else precond,
                              inner_relax=relax, inner_eps_max=1e-2,
                              variant=P.SHK_GMRES if variant is None else variant)
    nf = len(w.sigma)
    ws = torch.empty(P.shk_workspace_bytes(gp, prm, nf, 1), dtype=torch.uint8, device="cuda")
    b = torch.from_numpy(w.b[:, 0]).cuda()[None, :].contiguous()
    x = torch.empty((1, nf, gp.n), dtype=torch.complex128, device="cuda")
    for _ in range(warmup):
        P.fgmres_sh_solve(gp, prm, w.sigma, b, x=x, workspace=ws)
    torch.cuda.synchronize()
    if profile:
        P.shk_profile_enable(True)
    per = []
    worst = 0.0
    ok = True
    inner = outer = sweeps = 0
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        _, st = P.fgmres_sh_solve(gp, prm, w.sigma, b, x=x, workspace=ws)
        e1.record()
        e1.synchronize()
        per.append(e0.elapsed_time(e1))
        worst = max(worst, float(st["true_relres"].max()))
        ok &= bool((st["status"] == P.SHK_CONVERGED).all()) and worst <= w.tol
        inner = int(st["inner_its"][0, 0])
        outer = int(st["outer_its"].max())
        sweeps = int(st["refine_sweeps"].max())
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = ev0.elapsed_time(ev1)
    prof = None
    if profile:
        prof = P.shk_profile_read()
        P.shk_profile_enable(False)
    return dict(total_ms=total_ms, wall_s=wall, per_ms=per, worst=worst, ok=ok, inner=inner, outer=outer,
                sweeps=sweeps, prof=prof)


def roofline(prof, traffic_file, label, unit):
    """HBM roofline of one unit of work (a kernel launch, or one inner
    iteration made of several launches) from the library's live timing:
    (units, milliseconds, algorithmic bytes) summed over the timed region.
    The measured traffic is taken from the committed counter summary only
    while the kernel sources it was taken from are unchanged."""
    units, ms, nbytes = prof
    if units <= 0:
        return None
    avg_s = ms / units / 1e3
    achieved = nbytes / units / avg_s / 1e9
    r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": label, "per": unit,
         f"avg_{unit}_us": round(ms / units * 1e3, 3), f"{unit}s": units,
         f"algorithmic_bytes_per_{unit}": round(nbytes / units)}
    tfile = os.path.join(ROOT, "profiles", traffic_file)
    if os.path.exists(tfile):
        t = json.load(open(tfile))
        if t.get("kernel_source_digest") == kernel_source_digest():
            r["traffic"] = t.get(f"traffic_bytes_per_{unit}")
    return r


def sensitivity_bench(P, torch, w, make, n_src=8, n_rec=8, reps=5):
    """Sensitivities (section 5, eq. sensitivity) from one batched solve of the
    256x256 workload: its first n_src well sources as forward solutions and its
    first n_rec receiver vectors as adjoint solutions, J in complex64.  Timed
    with events on the stream the kernel runs on; roofline against HBM."""
    gp = make(w)
    prm, keep = P.make_params(w.tau_seq, m_restart=w.m_restart, max_restarts=20, max_refine=4, tol=w.tol,
                              eps_inner=w.eps_inner, precision=P.SHK_MIXED, inner_precond=P.SHK_PRECOND_MULTIGRID)
    b = torch.from_numpy(np.ascontiguousarray(w.b.T)).cuda()
    x, st = P.fgmres_sh_solve(gp, prm, w.sigma, b)
    nw = len(w.extra["wells"])
    phi = x[:n_src].contiguous()
    psi = x[nw:nw + n_rec].contiguous()
    n, nf = gp.n, len(w.sigma)
    J = torch.empty(n * nf * n_src * n_rec, dtype=torch.complex64, device="cuda")
    P.shk_sensitivity(gp, phi, psi, J, nf, n_src, n_rec)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        P.shk_sensitivity(gp, phi, psi, J, nf, n_src, n_rec)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    # algorithmic bytes: J written once, phi and psi read once, faces and K read once
    nbytes = n * nf * n_src * n_rec * 8 + n * nf * (n_src + n_rec) * 16 + n * (2 * 8 + 8)
    gbs = nbytes / (ms / 1e3) / 1e9
    out = {"workload": f"2-D FV 256x256, {nf} shifts, {n_src} sources x {n_rec} receivers from the 64-rhs solve",
           "entries": n * nf * n_src * n_rec, "dtype": "c64", "ms": round(ms, 3),
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gbs / HBM_PEAK_GBS, 4), "kernel": "k_sensitivity<float, 4, 4>",
                        "algorithmic_bytes_per_launch": nbytes}}
    gp.close()
    return out


MFMA_PEAK_TFLOPS = {"fp32": 157.3, "fp64": 78.6}


def block_gs_roofline(prof, precision_name):
    """Matrix-core roofline of the block Gram-Schmidt of the shared block basis
    (two projections V^H W and two updates W -= V C per block step, timed
    live with HIP events on the solve stream): achieved flops per second
    against the dense MFMA peak of its arithmetic type."""
    calls, ms, flops = prof
    if calls <= 0 or ms <= 0:
        return None
    tf = flops / (ms / 1e3) / 1e12
    peak = MFMA_PEAK_TFLOPS[precision_name]
    return {"bound": "mfma", "achieved": round(tf, 2), "peak": peak, "unit": "TFLOP/s", "frac": round(tf / peak, 4),
            "traffic": None, "kernel": f"k_blk_gram + k_blk_reduce + k_blk_update ({precision_name} 16x16x4 MFMA)",
            "calls": calls, "avg_call_us": round(ms / calls * 1e3, 2), "flops_per_call": round(flops / calls)}


def time_batched(P, torch, w, make, precision, single_rhs_sample=0, label=None, rhs_mode=None, m_restart=None):
    """One solve of a multi-rhs workload (all rhs in lockstep); with
    single_rhs_sample > 0, instead that many rhs solved one at a time and the
    rate scaled to all of them (multigrid-preconditioned inner solves).
    Returns shifted solves/s and the worst true relative residual; with a
    label, also the HBM roofline of one multigrid-COCG inner iteration at this
    workload, from one more solve with the library's per-iteration events
    (kept out of the timed solve)."""
    gp = make(w)
    block = rhs_mode == P.SHK_RHS_BLOCK
    prm, keep = P.make_params(w.tau_seq, m_restart=m_restart or w.m_restart, max_restarts=20, max_refine=4,
                              tol=w.tol, eps_inner=w.eps_inner, precision=precision,
                              inner_precond=P.SHK_PRECOND_MULTIGRID,
                              rhs_mode=P.SHK_RHS_LOCKSTEP if rhs_mode is None else rhs_mode)
    nf, nr = len(w.sigma), w.b.shape[1]
    cols = list(range(single_rhs_sample)) if single_rhs_sample else [list(range(nr))]
    worst, ok, total = 0.0, True, 0.0
    for c in cols:
        idx = [c] if single_rhs_sample else c
        b = torch.from_numpy(np.ascontiguousarray(w.b[:, idx].T)).cuda()
        P.fgmres_sh_solve(gp, prm, w.sigma, b)          # warm-up (allocations, code load)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _, st = P.fgmres_sh_solve(gp, prm, w.sigma, b)
        e1.record()
        e1.synchronize()
        total += e0.elapsed_time(e1) / 1e3
        worst = max(worst, float(st["true_relres"].max()))
        ok &= bool((st["status"] == P.SHK_CONVERGED).all())
    solves = nf * (len(cols) if single_rhs_sample else nr)
    out = {"solves_per_s": round(solves / total, 1), "ms": round(total * 1e3, 1), "converged": ok,
           "max_true_relres": worst, "outer_steps": int(st["outer_its"].max()),
           "inner_iterations": int(st["inner_its"][0, 0]), "refine_sweeps": int(st["refine_sweeps"].max())}
    if block:
        out["m_restart"] = prm.m_restart
    if label is not None:
        P.shk_profile_enable(True)
        P.fgmres_sh_solve(gp, prm, w.sigma, b)
        torch.cuda.synchronize()
        prof = P.shk_profile_read()
        bprof = P.shk_profile_read_block()
        P.shk_profile_enable(False)
        tfile = "none"
        if precision == P.SHK_MIXED and not block and not single_rhs_sample:
            tfile = {65536: "traffic_mg_iteration_256x256_64rhs.json",
                     2097152: "traffic_mg_iteration_128cubed_8rhs.json"}.get(gp.n, "none")
        out["roofline_iteration"] = roofline(prof, tfile, label, "iteration")
        if block:
            out["roofline_block_gs"] = block_gs_roofline(bprof, "fp32" if precision == P.SHK_MIXED else "fp64")
    gp.close()
    return out


def server_bench(P, torch, n_req=48, slots=4, budget_gb=200.0):
    """Serving workload: the first n_req requests of the seeded Poisson trace
    (20 requests/s; each a 2-D grid of 128^2, 256^2 or 512^2 with its own field,
    5-200 shifts, 1-16 point sources), replayed in real time.  The server (one
    device arena of min(budget_gb, 70% of free HBM), slots on their own
    streams, each request's right-hand sides in lockstep on complex64 vectors,
    multigrid inner solves, target 1e-6 after refinement) returns the solution
    at the source cells (SHK_OUT_ROWS).  Baseline: the same arrivals served
    one request at a time in arrival order by the plain FP64 solver, one
    right-hand side at a time.  Latency = completion - arrival."""
    import synth
    trace = synth.server_trace(max_requests=n_req)
    works = [synth.request_workload(r) for r in trace]
    rows = [np.array([int(np.argmax(np.abs(w.b[:, r]))) for r in range(w.b.shape[1])], dtype=np.int64)
            for w in works]
    solves = sum(len(w.sigma) * w.b.shape[1] for w in works)
    span = trace[-1].arrival - trace[0].arrival
    free, _total = torch.cuda.mem_get_info()
    budget = int(min(budget_gb * 1e9, 0.7 * free)) & ~255
    arena = torch.empty(budget, dtype=torch.uint8, device="cuda")
    keep = []
    srv = P.Server(budget, max_slots=slots, arena=arena)
    t0 = time.perf_counter()
    tickets = []
    for req, w, rw in zip(trace, works, rows):
        delay = req.arrival - trace[0].arrival - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        prm, k = P.make_params(w.tau_seq, m_restart=50, max_refine=4, tol=1e-6, eps_inner=1e-6,
                               precision=P.SHK_MIXED, inner_precond=P.SHK_PRECOND_MULTIGRID,
                               output=P.SHK_OUT_ROWS, out_rows=rw)
        keep.append(k)
        tickets.append(srv.submit(w.cell_K, w.sigma, w.b, prm, keep_solution=True))
    srv.drain()
    lat, ok, worst, t_first, t_last, errors = [], True, 0.0, None, 0.0, 0
    for t, w in zip(tickets, works):
        res, x, st = srv.poll(t, want_solution=True)
        lat.append((res["t_done"] - res["t_arrival"]) * 1e3)
        errors += res["error"] != 0
        ok &= res["error"] == 0 and res["n_converged"] == len(w.sigma) * w.b.shape[1]
        worst = max(worst, res["max_true_relres"])
        t_first = res["t_arrival"] if t_first is None else min(t_first, res["t_arrival"])
        t_last = max(t_last, res["t_done"])
    # the same requests submitted at once: the rate the server sustains when
    # arrivals never leave it idle
    t_b0 = srv.clock()
    bt = []
    for w, rw in zip(works, rows):
        prm, k = P.make_params(w.tau_seq, m_restart=50, max_refine=4, tol=1e-6, eps_inner=1e-6,
                               precision=P.SHK_MIXED, inner_precond=P.SHK_PRECOND_MULTIGRID,
                               output=P.SHK_OUT_ROWS, out_rows=rw)
        keep.append(k)
        bt.append(srv.submit(w.cell_K, w.sigma, w.b, prm, keep_solution=False))
    srv.drain()
    b_done = max(srv.poll(t)[0]["t_done"] for t in bt)
    burst = {"solves_per_s": round(solves / (b_done - t_b0), 1), "makespan_s": round(b_done - t_b0, 3),
             "requests_per_s": round(len(works) / (b_done - t_b0), 1)}
    srv.close()
    del arena
    torch.cuda.empty_cache()
    makespan = t_last - t_first
    server = {"solves_per_s": round(solves / makespan, 1), "makespan_s": round(makespan, 3),
              "p50_ms": round(percentile(lat, 0.5), 1), "p99_ms": round(percentile(lat, 0.99), 1),
              "converged": bool(ok), "request_errors": errors, "max_true_relres": worst, "slots": slots,
              "arena_gb": round(budget / 1e9, 1)}
    # sequential plain FP64, one rhs at a time, arrivals replayed
    gps = [P.Problem.fv2d(w.cell_K, w.Ss, w.h) for w in works]
    lat2, worst2, ok2 = [], 0.0, True
    t0 = time.perf_counter()
    busy_until = 0.0
    for req, w, gp in zip(trace, works, gps):
        arr = req.arrival - trace[0].arrival
        now = time.perf_counter() - t0
        if arr > now:
            time.sleep(arr - now)
        prm, k = P.make_params(w.tau_seq, m_restart=50, max_refine=4, tol=1e-6, eps_inner=1e-6,
                               precision=P.SHK_FP64, inner_precond=P.SHK_PRECOND_MULTIGRID)
        for r in range(w.b.shape[1]):
            b = torch.from_numpy(np.ascontiguousarray(w.b[:, r])).cuda()[None, :].contiguous()
            _, st = P.fgmres_sh_solve(gp, prm, w.sigma, b)
            worst2 = max(worst2, float(st["true_relres"].max()))
            ok2 &= bool((st["status"] == P.SHK_CONVERGED).all())
        torch.cuda.synchronize()
        done = time.perf_counter() - t0
        busy_until = done
        lat2.append((done - arr) * 1e3)
    for gp in gps:
        gp.close()
    seq = {"solves_per_s": round(solves / busy_until, 1), "makespan_s": round(busy_until, 3),
           "p50_ms": round(percentile(lat2, 0.5), 1), "p99_ms": round(percentile(lat2, 0.99), 1),
           "converged": bool(ok2), "max_true_relres": worst2}
    return {"workload": f"first {n_req} requests of the seeded Poisson trace (20 req/s over {span:.2f} s): 2-D grids "
                        f"128^2/256^2/512^2, 5-200 shifts, 1-16 rhs; {solves} shifted solves",
            "server_mixed_batched": server, "sequential_fp64_single_rhs": seq,
            "server_all_at_once": dict(burst, note="the same requests submitted together: sustainable rate"),
            "speedup_solves_per_s": round(server["solves_per_s"] / seq["solves_per_s"], 2),
            "saturated": bool(makespan > 1.2 * span),
            "note": "saturated means the makespan exceeds the trace span by 20%: arrivals outpace the GPU and "
                    "latency includes queueing; solves_per_s is then the sustainable rate"}


def cpu_baseline(w, seconds, gpu_outer_steps):
    """The CPU oracle (FGMRES-Sh, complex128, multigrid-COCG inner) on the same
    workload, bounded to a few outer steps; scaled to a full solve with the
    outer step count the GPU solve needed (refinement not counted)."""
    import numpy as np  # noqa: F401
    from oracle import Problem as OProblem, fgmres_sh
    op = OProblem.fv(w.cell_K, w.Ss, w.h)
    n_tau = len(w.tau_seq)
    steps = n_tau          # one step per preconditioner shift: the cycle's cost mix
    c0 = time.process_time()
    t0 = time.perf_counter()
    while True:
        fgmres_sh(op, w.b[:, 0], w.sigma, w.tau_seq, m_restart=w.m_restart, tol=w.tol, inner="mg",
                  eps=w.eps_inner, max_steps=steps)
        el = time.perf_counter() - t0
        if el >= 0.5 * seconds or steps >= 4 * n_tau:
            break
        steps += n_tau
        c0 = time.process_time()
        t0 = time.perf_counter()
    cpu = time.process_time() - c0
    per_step = el / steps
    est = per_step * max(gpu_outer_steps, 1)
    threads = max(1, int(round(cpu / el)))
    return {"value": len(w.sigma) / est, "unit": "shifted solves/s", "cores": threads, "kind": "oracle",
            "extrapolated": True,
            "sample": (f"{steps} outer steps (all {len(w.sigma)} shifts, multigrid-COCG inner to {w.eps_inner}) "
                       f"of the 512x512 workload in {el:.1f} s, extrapolated to the {gpu_outer_steps} outer steps "
                       f"of the GPU solve (refinement sweeps not counted)"),
            "host_cores_available": len(os.sched_getaffinity(0)),
            "direct": cpu_direct(w, max(2.0, 0.5 * seconds))}


def cpu_direct(w, seconds):
    """The sparse direct alternative: one SuperLU factorization and solve per
    shift (complex128, the oracle's exact solver), on the first shifts of the
    512x512 workload until about `seconds` have passed; every shift costs the
    same, so the rate is per shift measured, not extrapolated from a partial
    solve."""
    from oracle import Problem as OProblem, superlu_solve
    op = OProblem.fv(w.cell_K, w.Ss, w.h)
    b = w.b[:, 0]
    c0, t0 = time.process_time(), time.perf_counter()
    done = 0
    for sg in w.sigma:
        superlu_solve(op.shifted(sg), b)
        done += 1
        if time.perf_counter() - t0 >= seconds:
            break
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "shifted solves/s", "cores": max(1, int(round((time.process_time() - c0) / el))),
            "kind": "superlu (scipy splu, complex128)", "sample": f"{done} of {len(w.sigma)} shifts in {el:.1f} s"}


def phase_breakdown(P, torch, gp, w, precision, steps):
    """Where one solve's time goes, from the library's phase timer (HIP events
    at the phase boundaries on the solve stream, no per-iteration events), over
    `steps` solves after a warm-up; ms per solve."""
    prm, keep = P.make_params(w.tau_seq, m_restart=w.m_restart, max_restarts=20, max_refine=4, tol=w.tol,
                              eps_inner=w.eps_inner, precision=precision, inner_precond=P.SHK_PRECOND_MULTIGRID)
    nf = len(w.sigma)
    b = torch.from_numpy(w.b[:, 0]).cuda()[None, :].contiguous()
    x = torch.empty((1, nf, gp.n), dtype=torch.complex128, device="cuda")
    ws = torch.empty(P.shk_workspace_bytes(gp, prm, nf, 1), dtype=torch.uint8, device="cuda")
    P.fgmres_sh_solve(gp, prm, w.sigma, b, x=x, workspace=ws)
    torch.cuda.synchronize()
    P.shk_profile_enable(False, phases=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        P.fgmres_sh_solve(gp, prm, w.sigma, b, x=x, workspace=ws)
    e1.record()
    e1.synchronize()
    ph = P.shk_profile_read_phases()
    P.shk_profile_enable(False)
    total = e0.elapsed_time(e1) / steps
    out = {k: round(v / steps, 3) for k, v in ph.items() if v > 0}
    out["outside the solves' marks"] = round(total - sum(ph.values()) / steps, 3)
    out["ms_per_solve"] = round(total, 3)
    return out


def graph_ab(P, torch, gp, w, steps, warmup):
    """The 512x512 mixed solve with the inner iterations replayed from
    captured HIP graphs and launched one by one (the class's other settings
    unchanged), alternated twice; the class's setting is restored after."""
    prm, keep = P.make_params(w.tau_seq, m_restart=w.m_restart, precision=P.SHK_MIXED,
                              inner_precond=P.SHK_PRECOND_MULTIGRID)
    key = P.shk_tune_class(gp, prm, 1)
    was = P.shk_tune_get(key, "graph")
    ms = {0: [], 1: []}
    try:
        for g in (0, 1, 0, 1):
            P.shk_tune_set(key, "graph", g)
            r = time_path(P, torch, gp, w, P.SHK_MIXED, steps, warmup)
            ms[g].append(r["total_ms"] / steps)
    finally:
        P.shk_tune_set(key, "graph", was)
    off, on = float(np.mean(ms[0])), float(np.mean(ms[1]))
    return {"ms_per_solve_launched": round(off, 3), "ms_per_solve_graph": round(on, 3),
            "saving_frac": round((off - on) / off, 4), "runs": ms}


def autotune_bench(P, torch, path, reps=2):
    """Runs the autotuner on the benchmark workloads (both precisions) and
    writes the tuning cache to path."""
    import synth
    from paper_1212_3660_amd import autotune as T
    mk2 = lambda w: P.Problem.fv2d(w.cell_K, w.Ss, w.h)
    mk3 = lambda w: P.Problem.fv3d(w.cell_K, w.Ss, w.h)
    jobs = [("2-D FV 512x512, 1 rhs", synth.config2(n_grid=512), mk2, True),
            ("2-D FV 256x256, 64 rhs", synth.config3(), mk2, False),
            ("3-D FV 128^3, 8 rhs", synth.config4(), mk3, False)]
    entries = []
    for name, w, mk, one in jobs:
        gp = mk(w)
        bcols = w.b[:, :1] if one else w.b
        b = torch.from_numpy(np.ascontiguousarray(bcols.T)).cuda()
        for prec, pname in ((P.SHK_MIXED, "mixed"), (P.SHK_FP64, "fp64")):
            kw = dict(taus=w.tau_seq, m_restart=w.m_restart, max_restarts=20, max_refine=4, tol=w.tol,
                      eps_inner=w.eps_inner, precision=prec, inner_precond=P.SHK_PRECOND_MULTIGRID)
            print(f"[tune] {name}, {pname}", flush=True)
            e = T.tune(gp, w.sigma, b, kw, reps=reps, log=lambda m: print(m, flush=True),
                       workload=f"{name}, {pname}")
            print(json.dumps(e), flush=True)
            entries.append(e)
        gp.close()
    T.save(entries, path, device=torch.cuda.get_device_name(0))
    return entries


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the batched 256x256 / 128^3 workloads")
    ap.add_argument("--grid", type=int, default=512)
    ap.add_argument("--single-solve", choices=["mixed", "fp64"], default=None,
                    help="run one solve of the workload and exit (for profiler counter passes)")
    ap.add_argument("--precond", choices=["multigrid", "jacobi"], default="multigrid",
                    help="inner preconditioner of --single-solve")
    ap.add_argument("--solves", type=int, default=1,
                    help="solves --single-solve runs back to back (the first one cold)")
    ap.add_argument("--sensitivity-only", action="store_true",
                    help="run only the sensitivity measurement of the 256x256 workload and exit (profiler passes)")
    ap.add_argument("--batched-only", choices=["2d", "3d", "2d-block", "3d-block"], default=None,
                    help="run only the mixed batched 256x256 x 64 rhs (2d) or 128^3 x 8 rhs (3d) workload, with "
                         "independent bases or the shared block basis (-block), and exit (profiler passes)")
    ap.add_argument("--server-only", action="store_true",
                    help="run only the serving workload (trace replay) and exit")
    ap.add_argument("--no-server", action="store_true", help="skip the serving workload")
    ap.add_argument("--autotune", action="store_true",
                    help="run the autotuner on the benchmark workloads, write the tuning cache and exit")
    ap.add_argument("--tune-cache", default=None,
                    help="cache file --autotune writes (default: the packaged paper_1212_3660_amd/tune_cache.json)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="copy MIB mebibytes device-to-device with a plain copy kernel and exit "
                         "(calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the solver's per-GPU share is a whole "
              f"request or right-hand-side block, so N GPUs would run N independent copies", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    # every solve on a stream of its own (graph capture needs a stream other
    # than the legacy default one); torch's events record on it too
    with torch.cuda.stream(torch.cuda.Stream()):
        run(a)


def run(a):
    import torch
    import paper_1212_3660_amd as P
    import synth
    if a.autotune:
        autotune_bench(P, torch, a.tune_cache or P.autotune.CACHE)
        return
    if a.batched_only:
        if a.batched_only.startswith("2d"):
            wb, mk, name = synth.config3(), (lambda w: P.Problem.fv2d(w.cell_K, w.Ss, w.h)), "2-D FV 256x256, 64 rhs"
        else:
            wb, mk, name = synth.config4(), (lambda w: P.Problem.fv3d(w.cell_K, w.Ss, w.h)), "3-D FV 128^3, 8 rhs"
        blk = a.batched_only.endswith("block")
        r = time_batched(P, torch, wb, mk, P.SHK_MIXED, label=f"multigrid-COCG inner iteration, {name}, complex64",
                         rhs_mode=P.SHK_RHS_BLOCK if blk else None, m_restart=BLOCK_M if blk else None)
        name += ", shared block basis" if blk else ""
        print(json.dumps({"workload": name, **r}), flush=True)
        return
    if a.copy_calibration:
        src = torch.ones(a.copy_calibration << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4}), flush=True)
        return
    if a.server_only:
        print(json.dumps(server_bench(P, torch)), flush=True)
        return
    if a.sensitivity_only:
        print(json.dumps(sensitivity_bench(P, torch, synth.config3(), lambda w: P.Problem.fv2d(w.cell_K, w.Ss, w.h))),
              flush=True)
        return
    w = synth.config2(n_grid=a.grid)
    gp = P.Problem.fv2d(w.cell_K, w.Ss, w.h)
    if a.single_solve:
        prec = P.SHK_MIXED if a.single_solve == "mixed" else P.SHK_FP64
        pc = P.SHK_PRECOND_MULTIGRID if a.precond == "multigrid" else P.SHK_PRECOND_JACOBI
        r = time_path(P, torch, gp, w, prec, max(1, a.solves), 0, profile=False, precond=pc)
        print(json.dumps({"single_solve": a.single_solve, "precond": a.precond, "ms": r["total_ms"],
                          "ms_each": [round(v, 3) for v in r["per_ms"]], "inner_iterations": r["inner"],
                          "converged": r["ok"]}), flush=True)
        return
    # the inner-iteration kernel is timed inside the timed region itself
    mixed = time_path(P, torch, gp, w, P.SHK_MIXED, a.steps, a.warmup, profile=True)
    fp64 = time_path(P, torch, gp, w, P.SHK_FP64, a.steps, a.warmup, profile=False)
    # the same solves with the Jacobi-preconditioned inner COCG (its one
    # iteration kernel timed as well)
    jac = {"mixed": time_path(P, torch, gp, w, P.SHK_MIXED, a.steps, a.warmup, profile=True,
                              precond=P.SHK_PRECOND_JACOBI),
           "fp64": time_path(P, torch, gp, w, P.SHK_FP64, a.steps, a.warmup, profile=False,
                             precond=P.SHK_PRECOND_JACOBI)}
    # the same workload with the relaxed inner tolerance (an option, not the
    # configuration the metric is quoted on: its inner tolerance is fixed)
    relaxed = time_path(P, torch, gp, w, P.SHK_MIXED, a.steps, a.warmup, profile=False, relax=0.1)
    # the FOM projected problem (Algorithm 4, FOM) on the same workload
    fom = time_path(P, torch, gp, w, P.SHK_MIXED, a.steps, a.warmup, profile=False, variant=P.SHK_FOM)
    nf = len(w.sigma)
    ms_step = mixed["total_ms"] / a.steps
    value = nf * a.steps / (mixed["total_ms"] / 1e3)
    fp64_value = nf * a.steps / (fp64["total_ms"] / 1e3)
    # Roofline unit: one multigrid-COCG inner iteration (the step fused with
    # the first restriction, the V-cycle's other k_mg_down / k_mg_tail /
    # k_mg_up launches, k_cgmg_post), timed
    # with HIP events on the solver's stream around every chunk of iterations
    # inside the timed region; no single launch of it dominates.
    roof = roofline(mixed["prof"], "traffic_mg_iteration_512x512.json",
                    "multigrid-COCG inner iteration, mixed path: k_cgmg_step_down (step fused with the finest "
                    "restriction), the middle restrictions (k_mg_down_chain2d), k_mg_tail, the middle "
                    "prolongations (k_mg_up_chain2d), the finest k_mg_up, k_cgmg_post (6 launches; 10 without "
                    "the chains)", "iteration")
    roof_jac = roofline(jac["mixed"]["prof"], "traffic_cg_step_512x512.json",
                        "k_cg_step<Op2D<float>, float, ...> (Jacobi-COCG iteration, mixed path)", "launch")
    out = {"metric": METRIC, "value": round(value, 2), "unit": "shifted solves/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "c64+f64", "data": "synthetic",
           "config": {"workload": f"2-D FV {a.grid}x{a.grid}, {nf} shifts (periods 5..5000 s), 1 point source, "
                                  "tau cyclic {i w20, i w100, i w180}, inner COCG 1e-6, restart 50, target 1e-6",
                      "inner_preconditioner": "geometric multigrid V(1,1), damped Jacobi smoothing",
                      "n_shifts": nf, "n_rhs": 1, "unknowns": gp.n},
           "p50_ms": round(percentile(mixed["per_ms"], 0.5), 3), "p99_ms": round(percentile(mixed["per_ms"], 0.99), 3),
           "converged": mixed["ok"], "max_true_relres": mixed["worst"],
           "inner_iterations": mixed["inner"], "outer_steps": mixed["outer"], "refine_sweeps": mixed["sweeps"],
           "fp64": {"value": round(fp64_value, 2), "ms_per_step": round(fp64["total_ms"] / a.steps, 3),
                    "p50_ms": round(percentile(fp64["per_ms"], 0.5), 3),
                    "p99_ms": round(percentile(fp64["per_ms"], 0.99), 3), "converged": fp64["ok"],
                    "max_true_relres": fp64["worst"], "inner_iterations": fp64["inner"],
                    "outer_steps": fp64["outer"], "refine_sweeps": fp64["sweeps"]},
           "jacobi_inner": {name: {"value": round(nf * a.steps / (r["total_ms"] / 1e3), 2),
                                   "ms_per_step": round(r["total_ms"] / a.steps, 3), "converged": r["ok"],
                                   "max_true_relres": r["worst"], "inner_iterations": r["inner"]}
                            for name, r in jac.items()},
           "fom_variant": {"value": round(nf * a.steps / (fom["total_ms"] / 1e3), 2),
                           "ms_per_step": round(fom["total_ms"] / a.steps, 3), "converged": fom["ok"],
                           "max_true_relres": fom["worst"], "inner_iterations": fom["inner"],
                           "outer_steps": fom["outer"], "refine_sweeps": fom["sweeps"]},
           "relaxed_inner": {"inner_relax": 0.1, "inner_eps_max": 1e-2,
                             "value": round(nf * a.steps / (relaxed["total_ms"] / 1e3), 2),
                             "ms_per_step": round(relaxed["total_ms"] / a.steps, 3), "converged": relaxed["ok"],
                             "max_true_relres": relaxed["worst"], "inner_iterations": relaxed["inner"],
                             "outer_steps": relaxed["outer"], "refine_sweeps": relaxed["sweeps"]},
           "roofline": roof, "roofline_jacobi_step": roof_jac, "cpu_baseline": None}
    out["phases"] = {"mixed": phase_breakdown(P, torch, gp, w, P.SHK_MIXED, a.steps),
                     "fp64": phase_breakdown(P, torch, gp, w, P.SHK_FP64, a.steps)}
    out["captured_iterations"] = graph_ab(P, torch, gp, w, a.steps, a.warmup)
    tuned = [e["workload"] for e in P.autotune.load(apply=False)]
    out["tuning"] = {"cache": "paper_1212_3660_amd/tune_cache.json", "classes": tuned}
    if not a.no_extra:
        # the batched workloads: 256x256 with 32 well sources + 32 adjoint
        # receiver vectors, and 128^3 with 8 sources; mixed and FP64 paths in
        # lockstep over the rhs, and the 256x256 FP64 path one rhs at a time
        w3 = synth.config3()
        mk2 = lambda w: P.Problem.fv2d(w.cell_K, w.Ss, w.h)
        mk3 = lambda w: P.Problem.fv3d(w.cell_K, w.Ss, w.h)
        out["batched"] = {
            "2-D FV 256x256, 50 shifts, 64 rhs": {
                "mixed_batched": time_batched(P, torch, w3, mk2, P.SHK_MIXED,
                                              label="multigrid-COCG inner iteration, 64 lanes, complex64"),
                "mixed_block": time_batched(P, torch, w3, mk2, P.SHK_MIXED, rhs_mode=P.SHK_RHS_BLOCK,
                                            m_restart=BLOCK_M,
                                            label="multigrid-COCG inner iteration, 64 lanes, complex64"),
                "fp64_batched": time_batched(P, torch, w3, mk2, P.SHK_FP64,
                                             label="multigrid-COCG inner iteration, 64 lanes, complex128"),
                "fp64_block": time_batched(P, torch, w3, mk2, P.SHK_FP64, rhs_mode=P.SHK_RHS_BLOCK,
                                           m_restart=BLOCK_M,
                                           label="multigrid-COCG inner iteration, 64 lanes, complex128"),
                "fp64_single_rhs": dict(time_batched(P, torch, w3, mk2, P.SHK_FP64, single_rhs_sample=4),
                                        sample="4 of the 64 rhs solved one at a time, rate over those")},
        }
        out["sensitivity"] = sensitivity_bench(P, torch, w3, mk2)
        w4 = synth.config4()
        out["batched"]["3-D FV 128^3, 100 shifts, 8 rhs"] = {
            "mixed_batched": time_batched(P, torch, w4, mk3, P.SHK_MIXED,
                                          label="multigrid-COCG inner iteration, 8 lanes, complex64"),
            "mixed_block": time_batched(P, torch, w4, mk3, P.SHK_MIXED, rhs_mode=P.SHK_RHS_BLOCK, m_restart=BLOCK_M,
                                        label="multigrid-COCG inner iteration, 16 lanes (8 padded), complex64"),
            "fp64_batched": time_batched(P, torch, w4, mk3, P.SHK_FP64,
                                         label="multigrid-COCG inner iteration, 8 lanes, complex128")}
    if not a.no_server:
        out["serving"] = server_bench(P, torch)
    if not a.no_cpu:
        try:
            out["cpu_baseline"] = cpu_baseline(w, a.cpu_seconds, mixed["outer"])
        except Exception as e:  # the GPU numbers stand on their own
            out["cpu_baseline"] = {"error": str(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
