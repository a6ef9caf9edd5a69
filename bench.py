#!/usr/bin/env python3
"""Throughput of the steady phonon-BTE transport step on one MI355X.

Workload: 2D 1 um x 1 um square, 256 x 256 cells, 20 seeded bands
(tau log-uniform in [1e-12, 1e-9] s), 128 directions (2 polar x 8 azimuthal
nodes per octant), heat-sink edge at 300 K, three diffuse edges, Gaussian
volumetric source (sigma 50 nm, 1e17 W/m^3) at the centre; synthetic
scheme.  Inputs are synthetic (seeded), resident in HBM before timing.

A step is one source iteration of the steady solve: diffuse-wall inflow,
the transport sweep over every (cell, direction, band), FP64 moments, the
CG synthetic correction and the convergence check.  value = solid cells x
directions x bands x steps / wall time of the timed steps, FP32 storage of
the energy deviation with FP64 moments.  The FP64 path is timed the same
way, and both are run to convergence to report their relative difference.

--workload transient3d times the explicit transient step instead: 64^3
cube of (2 um)^3, 40 bands, 128 directions, MC limiter, dt = 0.5 ps, laser
pulse; a step is one explicit step of every (cell, direction, band).

--workload porous2d_batch solves the batch of 64 porous films (sides 32 to
256 cells, 64 directions, 20 bands) to convergence in one problem and
reports k_eff per film; --workload porous3d_adjoint solves the 48^3 porous
cube (96 directions, 40 bands, per-cell gamma) and its adjoint d k_eff /
d gamma; --workload tadjoint3d runs the transient adjoint of 500 explicit
steps on a 32^3 cube with checkpoints every 50 steps; --workload interface2d
solves two materials joined by the interfacial boundary condition (two
128 x 256 halves of a 1 um square, 20 bands, 128 directions, walls at
301 K / 299 K) to convergence and reports the interface conductance.

--copy-calibration runs a plain 2 GiB device copy (for scaling HBM counters).

Prints one JSON line.  --gpus N > 1 is not supported (one GPU only).
"""
import hashlib
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# sources each measured kernel is built from (the committed counter summary
# is used only while their hash matches)
# (bte_api.cpp builds the work-item order, which decides the L2 reuse)
KERNEL_SOURCES = {
    "k_sweep2d<float,0>": ("bte_sweep2d.hip", "bte_tilelds.h", "bte_tile.h", "bte_stencil.h", "bte_internal.h",
                           "bte_api.cpp"),
    "k_transient3d<float,1>": ("bte_transient3d.hip", "bte_tilelds.h", "bte_tile.h", "bte_stencil.h",
                               "bte_internal.h", "bte_api.cpp"),
    "k_sweep3d<float,0>": ("bte_sweep3d.hip", "bte_col3d.h", "bte_tilelds.h", "bte_tile.h", "bte_stencil.h",
                           "bte_internal.h", "bte_api.cpp"),
}
BYTES_PER_UPDATE = {0: 8.0, 1: 16.0}   # read e^n + write e^{n+1}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_steps(B, prob, e, steps, init):
    prob.set_control(max_iter=steps, residual_temp=0.0, residual_flux=0.0)
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = prob.steady_solve(e, init=init, allow_not_converged=True)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, st


def host_cpu():
    """CPU model, sockets, physical cores and hardware threads of the host
    (lscpu), and the OpenMP threads the oracle runs with."""
    info = {}
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        kv = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        sockets = int(kv.get("Socket(s)", "0") or 0)
        cps = int(kv.get("Core(s) per socket", "0") or 0)
        info = dict(model=kv.get("Model name"), sockets=sockets, physical_cores=sockets * cps,
                    hardware_threads=int(kv.get("CPU(s)", "0") or 0))
    except Exception as ex:   # lscpu missing: report what Python knows
        info = dict(model=None, error=str(ex))
    info["affinity_cpus"] = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    info["omp_threads"] = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return info


def cpu_baseline(cfg, seconds_hint=30.0):
    """Oracle (FP64 C, OpenMP) on a bounded sample: three source iterations of
    the same workload (sweep, moments, synthetic correction), started from the
    heat-diffusion state (computed untimed)."""
    import numpy as np
    import oracle as O
    case = O.Case(cfg["geometry"], cfg["material"], P=cfg["P"])
    Td = O.diffusion_T(case, rtol=1e-10)
    e0 = (case.C[None, None, :] * Td[:, None, None] / (4 * np.pi) * np.ones((1, case.na, 1))).reshape(-1)
    del Td
    t0 = time.perf_counter()
    iters = 3
    e1, st = O.steady(case, scheme=1, tol_T=0.0, tol_q=0.0, max_iter=iters, cg_rtol=1e-6, e=e0)
    dt = time.perf_counter() - t0
    updates = case.nc * case.na * case.nl * iters
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=updates / dt, unit="cell*dir*band updates/s", cores=threads, kind="oracle", host=host_cpu(),
                sample="%d source iterations (sweep + FP64 moments + CG correction) of the 256x256 x 128 dir x "
                       "20 band workload, %.1f s" % (iters, dt))


def kernel_source_hash(kernel):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2306_14181_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(kernel, variant=None):
    """HBM bytes per launch unit of `kernel` from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the
    kernel sources changed since the counters were taken or (`variant`:
    tuning kind and tile shape) another variant was measured."""
    f = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        d = json.load(fh)
    r = d.get(kernel)
    if not r or r.get("source_hash") != kernel_source_hash(kernel):
        return None
    if variant is not None and (r.get("kind"), tuple(r.get("tile", ()))) != (variant[0], tuple(variant[1])):
        return None
    return r["bytes_per_unit"]


def tune_sweep(B, prob, e, reps, one_launch):
    """Time every 2D sweep candidate (tile shape x launch form) and keep the
    fastest; with one_launch False only the per-diagonal launch forms compete.
    Returns the entries of the two sweep kinds."""
    tune = [dict(x) for x in prob.autotune(reps=reps, scratch=e)
            if x["kind"] in (B.TUNE_SWEEP, B.TUNE_SWEEP_ONE_LAUNCH)]
    if not one_launch:
        tune = [x for x in tune if x["kind"] == B.TUNE_SWEEP]
        best = min(tune, key=lambda x: x["ms"])
        for x in tune:
            x["chosen"] = x is best
        prob.set_tiles(B.TUNE_SWEEP, best["tile"])
    for x in tune:
        x["kernel"] = sweep_kernel_name(B, x["kind"], tuple(x["tile"]))
        log("autotune %s: %.3f ms per sweep%s" % (x["kernel"], x["ms"], "  (kept)" if x["chosen"] else ""))
    return tune


def sweep_kernel_name(B, kind, tile):
    if kind == B.TUNE_SWEEP_ONE_LAUNCH:
        return "k_sweep2d, %d tile rows per wavefront, one launch per sweep" % tile[2]
    if tuple(tile[:2]) == (8, 8):
        return "k_sweep2d, %d tile rows per wavefront, one launch per tile diagonal" % tile[2]
    return "k_sweep_tile, %dx%d LDS tiles, one launch per tile diagonal" % tuple(tile[:2])


def copy_calibration():
    import torch
    n = 1 << 29   # 2 GiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "ms": dt * 1e3,
                      "GBs": 8 * n / dt / 1e9}), flush=True)


def bench_transient(args):
    import numpy as np
    import torch

    import bte_inputs as I
    from paper_2306_14181_amd import bte as B

    torch.cuda.set_device(0)
    n = args.n or 64
    cfg = I.cube3d_laser_case(n=n)
    P = torch.as_tensor(cfg["P"], device="cuda")
    res = {}
    for prec in ([B.F32] if args.no_fp64 else [B.F32, B.F64]):
        prob = B.Problem(cfg["geometry"], cfg["material"], dict(precision=prec, limiter=B.LIM_MC, dt=cfg["dt"]))
        prob.set_fields(P, None)
        e = prob.zeros()
        prob.transient_step(e, args.warmup, 0.0, cfg["pulse"])
        prob.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prob.transient_step(e, args.steps, args.warmup * cfg["dt"], cfg["pulse"])
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        st = prob.last_stats()
        upd = prob.n_unknowns
        T, _, _ = prob.moments(e)
        res[prec] = dict(t=t, st=st, upd=upd, T=T.cpu().numpy())
        log("transient prec %d: %d steps %.3f s, transport %.1f ms, walls %.1f ms, T_L %.1f ms"
            % (prec, args.steps, t, st["ms_sweep"], st["ms_walls"], st["ms_post"]))
        del prob, e
        torch.cuda.empty_cache()
    r = res[B.F32]
    value = r["upd"] * args.steps / r["t"]
    kern_ms = r["st"]["ms_sweep"] / args.steps
    achieved = BYTES_PER_UPDATE[B.F32] * r["upd"] / (kern_ms * 1e-3) / 1e9
    traffic = counter_traffic("k_transient3d<float,1>")
    out = {
        "metric": "cell*dir*band updates/s (FP32 state, FP64 moments) of explicit transient steps",
        "value": value, "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * r["t"] / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (e), f64 (moments)", "data": "synthetic (seeded bands, laser pulse)",
        "config": {"workload": "cube3d_laser: %d^3 cells, 2 um, 40 bands, 128 directions, MC limiter, dt 0.5 ps"
                   % n, "n": n},
        "roofline": {"bound": "hbm", "kernel": "k_transient3d<float,MC> (one launch per step)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "avg_launch_ms": kern_ms,
                     "bytes_per_launch": BYTES_PER_UPDATE[B.F32] * r["upd"]},
        "phase_ms_per_step": {"transport": kern_ms, "walls": r["st"]["ms_walls"] / args.steps,
                              "T_L": r["st"]["ms_post"] / args.steps},
    }
    if B.F64 in res:
        r64 = res[B.F64]
        T32, T64 = r["T"], r64["T"]
        out["fp64"] = {"value": r64["upd"] * args.steps / r64["t"], "ms_per_step": 1e3 * r64["t"] / args.steps,
                       "transport_GBs": BYTES_PER_UPDATE[B.F64] * r64["upd"] * args.steps
                       / (r64["st"]["ms_sweep"] * 1e-3) / 1e9}
        out["accuracy"] = {"T_rel_err_fp32_vs_fp64": float(np.abs(T32 - T64).max()
                                                           / max(np.abs(T64 - 300.0).max(), 1e-300)),
                           "after_steps": args.warmup + args.steps}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_transient()
    print(json.dumps(out), flush=True)


def cpu_baseline_transient():
    """Oracle transient steps on a bounded sample: 6 steps of the same physics
    on a 32^3 grid (one full 64^3 step takes minutes on the CPU)."""
    import numpy as np
    import bte_inputs as I
    import oracle as O
    cfg = I.cube3d_laser_case(n=32)
    case = O.Case(cfg["geometry"], cfg["material"], P=cfg["P"], limiter=cfg["limiter"])
    e = np.zeros(case.nc * case.na * case.nl)
    steps = 6
    t0 = time.perf_counter()
    O.transient(case, e, steps, cfg["dt"], 0.0, cfg["pulse"])
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=case.nc * case.na * case.nl * steps / dt, unit="cell*dir*band updates/s", cores=threads,
                kind="oracle", host=host_cpu(), sample="%d explicit steps of the laser workload on a 32^3 grid, %.1f s" % (steps, dt))


def bench_ttg(args):
    """Transient thermal grating at the paper's size (1000 cells, 512
    directions, gray, periodic) in three regimes, each run to t* = t / tau =
    2: explicit-step rate and the grating amplitude against the continuous
    gray solution."""
    import numpy as np
    import torch

    import bte_inputs as I
    from paper_2306_14181_amd import bte as B
    from tests.helpers import ttg_continuous_amplitude

    torch.cuda.set_device(0)
    x = (np.arange(1000) + 0.5) * 1e-9
    runs = []
    for xi in (0.1, 1.0, 10.0):
        cfg = I.ttg(xi)
        m = cfg["material"]
        steps = int(round(2.0 * cfg["tau"] / cfg["dt"]))
        ac = float(ttg_continuous_amplitude([2.0], m["v"][0], cfg["tau"], 1e-6)[0])
        for prec in ([B.F32] if args.no_fp64 else [B.F32, B.F64]):
            prob = B.Problem(cfg["geometry"], m, dict(precision=prec, limiter=B.LIM_NONE, dt=cfg["dt"]))
            prob.set_fields(None, None)
            e0 = (m["C"][0] * (cfg["T0"] - 300.0) / (4 * np.pi))[:, None] * np.ones(512)[None, :]
            e = torch.as_tensor(e0.reshape(-1), device="cuda").to(prob.dtype)
            w = prob.zeros()
            w.copy_(e)
            prob.transient_step(w, args.warmup)   # warm-up on a copy
            prob.set_timing(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            prob.transient_step(e, steps)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            st = prob.last_stats()
            T, _, _ = prob.moments(e)
            amp = 2.0 * float(np.mean((T.cpu().numpy() - 300.0) * np.cos(2 * np.pi * x / 1e-6)))
            runs.append(dict(xi=xi, prec=prec, steps=steps, t=t, kern_ms=st["ms_sweep"] / steps,
                             upd=prob.n_unknowns, amp=amp, cont=ac))
            log("ttg xi %.1f prec %d: %d steps %.3f s (%.1f us per step, transport %.1f us), A/A0 %.5f, "
                "continuous %.5f" % (xi, prec, steps, t, 1e6 * t / steps, 1e3 * st["ms_sweep"] / steps, amp, ac))
            del prob, e, w
    f32 = [r for r in runs if r["prec"] == B.F32]
    upd = sum(r["upd"] * r["steps"] for r in f32)
    tt = sum(r["t"] for r in f32)
    kern_ms = sum(r["kern_ms"] * r["steps"] for r in f32) / sum(r["steps"] for r in f32)
    achieved = BYTES_PER_UPDATE[B.F32] * f32[0]["upd"] / (kern_ms * 1e-3) / 1e9
    out = {
        "metric": "cell*dir*band updates/s (FP32 state, FP64 moments) of explicit transient steps",
        "value": upd / tt, "unit": "updates/s", "n_gpus": 1, "steps": sum(r["steps"] for r in f32),
        "warmup": args.warmup, "ms_per_step": 1e3 * tt / sum(r["steps"] for r in f32), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (e), f64 (moments)",
        "data": "synthetic (gray band, cosine grating)",
        "config": {"workload": "ttg1d: 1000 cells, one 1 um period, 512 directions, 1 band, xi 0.1 / 1 / 10 "
                   "to t* = 2, no limiter"},
        "roofline": {"bound": "hbm", "kernel": "k_transient_tile<float,1D,NONE> (one launch per step)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "avg_launch_ms": kern_ms,
                     "bytes_per_launch": BYTES_PER_UPDATE[B.F32] * f32[0]["upd"],
                     "note": "4 MB state: resident in L2, launch-latency bound"},
        "amplitude_at_t2": [{"xi": r["xi"], "precision": "f32" if r["prec"] == B.F32 else "f64",
                             "A_over_A0": r["amp"], "continuous": r["cont"]} for r in runs],
    }
    if not args.no_cpu_baseline:
        import oracle as O
        cfg = I.ttg(1.0)
        case = O.Case(cfg["geometry"], cfg["material"])
        e0 = (cfg["material"]["C"][0] * (cfg["T0"] - 300.0) / (4 * np.pi))[:, None] * np.ones(case.na)[None, :]
        n = 1000
        t0 = time.perf_counter()
        O.transient(case, e0.reshape(-1), n, cfg["dt"])
        dt = time.perf_counter() - t0
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        out["cpu_baseline"] = dict(value=case.nc * case.na * n / dt, unit="cell*dir*band updates/s", cores=threads,
                                   host=host_cpu(),
                                   kind="oracle", sample="%d explicit steps of the xi = 1 grating, %.1f s" % (n, dt))
    print(json.dumps(out), flush=True)


def bench_batch(args):
    """64 porous films in one problem, FP32, converged steady solve."""
    import numpy as np
    import torch
    import bte_inputs as I
    from paper_2306_14181_amd import bte as B
    torch.cuda.set_device(0)
    cfg = I.porous2d_batch_case()
    films, mat = cfg["films"], cfg["material"]
    prob = B.Problem(films, mat, dict(precision=B.F32, scheme=B.SYNTHETIC, limiter=cfg["limiter"],
                                      residual_temp=1e-6, residual_flux=1e-5, max_iter=args.max_iter,
                                      cg_rtol=1e-6, cg_max_iter=40))
    prob.set_persistent(not args.no_persistent)
    e = prob.zeros()
    tune = []
    if not args.no_autotune:
        # every sweep candidate (register tile with 2, 1, 4 rows per
        # wavefront, per-diagonal launches or one launch; LDS tiles) timed
        # on one sweep of all films, fastest kept
        tune = tune_sweep(B, prob, e, 2, not args.no_persistent)
        e.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = prob.steady_solve(e, init=True, allow_not_converged=True)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    k = prob.keff(e).cpu().numpy()
    solid = sum(int(np.count_nonzero(g["solid"])) for g in films)
    upd = st["updates"]   # converged films are no longer swept
    log("batch: %d films, %d cells (%d solid), %d iterations %.2f s, sweep %.0f ms, cg %.0f ms"
        % (len(films), prob.n_cells, solid, st["iters"], t, st["ms_sweep"], st["ms_cg"]))
    out = {"metric": "cell*dir*band updates/s of the batched steady solve (FP32 state, FP64 moments)",
           "value": upd / t, "unit": "updates/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f32 (e), f64 (moments, CG)",
           "data": "synthetic (seeded porous films)",
           "config": {"workload": "porous2d_batch: 64 films, sides 32-256, dx 1 um/256, 64 directions, 20 bands, minmod limiter",
                      "cells": prob.n_cells, "solid_cells": solid, "unknowns": prob.n_unknowns},
           "iterations": st["iters"], "converged": st["converged"], "eps_T": st["eps_T"], "eps_q": st["eps_q"],
           "solve_s": t,
           "ms_per_iteration": 1e3 * t / max(st["iters"], 1),
           "phase_ms_per_iteration": {kk: st[kk] / max(st["iters"], 1) for kk in ("ms_sweep", "ms_walls", "ms_post", "ms_cg")},
           "sweep_GBs": BYTES_PER_UPDATE[B.F32] * upd / (st["ms_sweep"] * 1e-3) / 1e9,
           "note": "updates counted per film until it converges (per-film masks); a film of n cells adds "
                   "n x 64 directions x 20 bands per iteration while it is swept",
           "keff": {"min": float(k.min()), "mean": float(k.mean()), "max": float(k.max())},
           "autotune": [{"tile": list(x["tile"]), "kernel": x["kernel"], "ms_per_sweep": x["ms"], "chosen": x["chosen"]}
                        for x in tune]}
    print(json.dumps(out), flush=True)


def bench_interface(args):
    """Two materials joined by the interfacial boundary condition: steady
    FP32 solve to convergence, the sweep roofline and the interface
    conductance q_x / (T just left of the interface - T just right of it)."""
    import numpy as np
    import torch
    import bte_inputs as I
    from paper_2306_14181_amd import bte as B
    torch.cuda.set_device(0)
    cfg = I.interface2d_case()
    geos, mats = cfg["geometries"], cfg["materials"]
    prob = B.Problem(geos, mats, dict(precision=B.F32, scheme=B.SYNTHETIC, limiter=cfg["limiter"],
                                      residual_temp=1e-6, residual_flux=1e-5, max_iter=args.max_iter,
                                      cg_rtol=1e-6, cg_max_iter=40),
                     geo_mat=cfg["geo_mat"], interfaces=cfg["interfaces"])
    prob.set_persistent(not args.no_persistent)
    e = prob.zeros()
    tune = []
    if not args.no_autotune:
        tune = tune_sweep(B, prob, e, 2, not args.no_persistent)
        e.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = prob.steady_solve(e, init=True, allow_not_converged=True)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    T, _, q = prob.moments(e)
    T, q = T.cpu().numpy(), q.cpu().numpy()
    nA, ny = geos[0]["n"][0], geos[0]["n"][1]
    nB = geos[1]["n"][0]
    TA = T[: nA * ny].reshape(ny, nA)
    TB = T[nA * ny:].reshape(ny, nB)
    qA = q[: nA * ny, 0].reshape(ny, nA)
    qB = q[nA * ny:, 0].reshape(ny, nB)
    dT = float(TA[:, -1].mean() - TB[:, 0].mean())
    qi = float(0.5 * (qA[:, -1].mean() + qB[:, 0].mean()))
    upd = st["updates"]
    sweep_ms = st["ms_sweep"] / max(st["iters"], 1)
    sweep_bytes = BYTES_PER_UPDATE[B.F32] * prob.n_cells * prob.n_dirs * prob.n_bands
    achieved = sweep_bytes / (sweep_ms * 1e-3) / 1e9
    kept = next((x for x in tune if x["chosen"]), None)
    log("interface2d: %d iterations %.2f s, sweep %.3f ms, G = %.4g W/m^2/K" % (st["iters"], t, sweep_ms, qi / dT))
    out = {"metric": "cell*dir*band updates/s of the steady solve of two materials joined by an interface",
           "value": upd / t, "unit": "updates/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "f32 (e), f64 (moments, CG)", "data": "synthetic (seeded bands, diffuse-mismatch-form beta)",
           "config": {"workload": "interface2d: 2 x (128 x 256) cells of a 1 um square, 20 bands, 128 directions, "
                                  "walls 301 K / 299 K, specular top and bottom", "unknowns": prob.n_unknowns},
           "iterations": st["iters"], "converged": st["converged"], "eps_T": st["eps_T"], "solve_s": t,
           "roofline": {"bound": "hbm", "kernel": kept["kernel"] if kept else "k_sweep2d", "achieved": achieved,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                        "avg_sweep_ms": sweep_ms, "bytes_per_sweep": sweep_bytes},
           "interface": {"q_x": qi, "T_left": float(TA[:, -1].mean()), "T_right": float(TB[:, 0].mean()),
                         "conductance_W_m2K": qi / dT,
                         "q_x_spread": float((max(qA.max(), qB.max()) - min(qA.min(), qB.min())) / abs(qi))},
           "autotune": [{"tile": list(x["tile"]), "kernel": x["kernel"], "ms_per_sweep": x["ms"],
                         "chosen": x["chosen"]} for x in tune]}
    print(json.dumps(out), flush=True)


def bench_adjoint(args):
    """48^3 porous cube: FP32 forward steady solve and the adjoint gradient."""
    import numpy as np
    import torch
    import bte_inputs as I
    from paper_2306_14181_amd import bte as B
    torch.cuda.set_device(0)
    cfg = I.porous3d_adjoint_case()
    g, mat = cfg["geometry"], cfg["material"]
    ctl = dict(precision=B.F32, scheme=B.SYNTHETIC, limiter=B.LIM_NONE, adjoint=True, residual_temp=1e-6,
               residual_flux=1e-5, max_iter=args.max_iter, cg_rtol=1e-6, cg_max_iter=40)
    prob = B.Problem(g, mat, ctl)
    prob.set_fields(None, torch.as_tensor(cfg["gamma"], device="cuda"))
    e = prob.zeros()
    tune = []
    if not args.no_autotune:
        # tile shape of the LDS-tile sweeps (forward and adjoint), chosen by timing every candidate
        tune = prob.autotune(reps=2, scratch=e)
        for x in tune:
            log("autotune %s tile %s: %.2f ms per sweep%s" % ("sweep" if x["kind"] == B.TUNE_SWEEP else "step",
                                                               "x".join(map(str, x["tile"])), x["ms"],
                                                               "  (kept)" if x["chosen"] else ""))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = prob.steady_solve(e, init=True, allow_not_converged=True)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    k = prob.keff(e).item()
    prob.set_control(**dict(ctl, residual_temp=1e-5))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grad, sa = prob.adjoint(e, allow_not_converged=True)
    torch.cuda.synchronize()
    ta = time.perf_counter() - t0
    gr = grad.cpu().numpy()
    upd = prob.n_unknowns
    # roofline of the transport sweeps: algorithmic bytes (read e^n + write
    # e^{n+1} of every solid cell, direction and band) over the device time
    # of one sweep (HIP events around the hyperplane launches on the stream)
    solid = int(np.asarray(g["solid"]).astype(bool).sum())
    sweep_bytes = BYTES_PER_UPDATE[B.F32] * solid * prob.n_dirs * prob.n_bands
    fwd_ms = st["ms_sweep"] / max(st["iters"], 1)
    adj_ms = sa["ms_sweep"] / max(sa["iters"], 1)
    roof = lambda ms: sweep_bytes / (ms * 1e-3) / 1e9
    log("adjoint3d: forward %d its %.2f s, adjoint %d sweeps %.2f s (residual %.1e)"
        % (st["iters"], tf, sa["iters"], ta, sa["eps_T"]))
    out = {"metric": "forward and adjoint steady solves of the porous cube (FP32 state)",
           "value": upd * (st["iters"] + sa["iters"]) / (tf + ta), "unit": "updates/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "f32 (e, psi), f64 (moments, CG, gradient)",
           "data": "synthetic (seeded spherical pores, gamma ~ U[0, 1e11] 1/s)",
           "config": {"workload": "porous3d_adjoint: 48^3 cells of (1 um)^3, porosity 0.2, 96 directions, 40 bands",
                      "unknowns": upd},
           "forward": {"iterations": st["iters"], "converged": st["converged"], "solve_s": tf,
                       "ms_sweep_per_iteration": st["ms_sweep"] / max(st["iters"], 1), "keff": k},
           "adjoint": {"sweeps": sa["iters"], "converged": sa["converged"], "relative_residual": sa["eps_T"],
                       "solve_s": ta, "ms_sweep_per_iteration": sa["ms_sweep"] / max(sa["iters"], 1)},
           "adjoint_over_forward_time": ta / tf,
           "roofline": {"bound": "hbm", "kernel": "k_sweep3d<float,NONE> (the hyperplane launches of one sweep)",
                        "achieved": roof(fwd_ms), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": roof(fwd_ms) / HBM_PEAK_GBS, "traffic": counter_traffic("k_sweep3d<float,0>"),
                        "avg_sweep_ms": fwd_ms, "launches_per_sweep": st["sweep_launches"] / max(st["iters"], 1),
                        "bytes_per_sweep": sweep_bytes, "solid_cells": solid},
           "adjoint_roofline": {"kernel": "k_sweep3d<float,NONE,ADJ> (transposed sweep)", "achieved": roof(adj_ms),
                                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": roof(adj_ms) / HBM_PEAK_GBS,
                                "avg_sweep_ms": adj_ms},
           "autotune": [{"tile": list(x["tile"]), "ms_per_sweep": x["ms"], "chosen": x["chosen"]} for x in tune],
           "grad": {"min": float(gr.min()), "max": float(gr.max()), "sum": float(gr.sum())}}
    print(json.dumps(out), flush=True)


def bench_mesh(args):
    """Steady FP32 source iterations on an unstructured hybrid mesh of
    triangles and quadrilaterals (least-squares gradients over the cells
    sharing a vertex, sweeps by upwind levels): updates/s over a fixed
    number of iterations, the level-sweep roofline, and the oracle on a
    bounded sample."""
    import numpy as np
    import torch
    import bte_inputs as I
    from paper_2306_14181_amd import bte as B
    torch.cuda.set_device(0)
    mesh = I.mesh2d(21, 128, 128, 1e-6, 1e-6, jitter=0.25, quad_frac=0.3)
    mat = dict(I.bands(np.random.default_rng(21), 20), n_theta=2, n_phi=8, Tref=300.0)
    iters = max(args.steps, 1)
    prob = B.MeshProblem(mesh, mat, dict(precision=B.F32, max_iter=iters, residual_temp=0.0))
    e = prob.zeros()
    prob.steady_solve(e, init=True, allow_not_converged=True)   # warm-up (the same iterations)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = prob.steady_solve(e, init=True, allow_not_converged=True)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    upd = st["updates"]
    sweep_ms = st["ms_sweep"] / st["iters"]
    # level sweep: read R and e, write de and e per update
    sweep_bytes = 4.0 * 4 * prob.n_unknowns
    achieved = sweep_bytes / (sweep_ms * 1e-3) / 1e9
    log("mesh2d: %d cells, %d levels, %d iterations %.3f s: sweep %.3f ms, gradient+walls+residual %.3f ms, "
        "moments %.3f ms per iteration" % (prob.n_cells, prob.n_levels, st["iters"], t, sweep_ms,
                                           st["ms_walls"] / st["iters"], st["ms_post"] / st["iters"]))
    out = {"metric": "cell*dir*band updates/s of steady source iterations on an unstructured 2D mesh",
           "value": upd / t, "unit": "updates/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "f32 (e), f64 (gradient arithmetic, moments)", "data": "synthetic (seeded hybrid mesh, bands)",
           "config": {"workload": "mesh2d: 128 x 128 jittered grid of a 1 um square, squares kept (30 %) or split "
                                  "into triangles, 128 directions, 20 bands, thermalizing x walls, specular y walls",
                      "cells": prob.n_cells, "levels": prob.n_levels, "iterations": st["iters"]},
           "ms_per_iteration": t / st["iters"] * 1e3,
           "phase_ms_per_iteration": {"sweep": sweep_ms, "gradient_walls_residual": st["ms_walls"] / st["iters"],
                                      "moments": st["ms_post"] / st["iters"]},
           "roofline": {"bound": "hbm", "kernel": "k_mesh_sweep_level<float> (the level launches of one sweep)",
                        "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                        "traffic": None, "avg_sweep_ms": sweep_ms, "launches_per_sweep": prob.n_levels,
                        "bytes_per_sweep": sweep_bytes}}
    if not args.no_cpu_baseline:
        from oracle import mesh as M
        small = I.mesh2d(21, 16, 16, 1e-6 / 8, 1e-6 / 8, jitter=0.25, quad_frac=0.3)
        case = M.MeshCase(small, mat)
        ec = case.zeros()
        t1 = time.perf_counter()
        ec = M.sweep(case, ec, M.moments(case, ec)[1] - case.Tref)
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": case.size / dt, "unit": "cell*dir*band updates/s", "cores": 1,
                               "kind": "oracle", "host": host_cpu(),
                               "sample": "1 source iteration (numpy, FP64, one thread) of a 16 x 16 version of the "
                                         "mesh with the same directions and bands, %.1f s" % dt}
    print(json.dumps(out), flush=True)


def bench_mesh3d(args):
    """Steady FP32 source iterations on a tetrahedral mesh (jittered cubes,
    six Kuhn tetrahedra each; least-squares gradients over the cells sharing
    a vertex): updates/s over a fixed number of iterations and the
    level-sweep roofline."""
    import numpy as np
    import torch
    import bte_inputs as I
    from paper_2306_14181_amd import bte as B
    torch.cuda.set_device(0)
    n = 32
    mesh = I.mesh3d(31, n, n, n, 1e-6, 1e-6, 1e-6, jitter=0.15)
    mat = dict(I.bands(np.random.default_rng(31), 20), n_theta=3, n_phi=4, Tref=300.0)
    iters = max(min(args.steps, 30), 1)
    prob = B.MeshProblem(mesh, mat, dict(precision=B.F32, max_iter=iters, residual_temp=0.0))
    e = prob.zeros()
    prob.steady_solve(e, init=True, allow_not_converged=True)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = prob.steady_solve(e, init=True, allow_not_converged=True)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    sweep_ms = st["ms_sweep"] / st["iters"]
    sweep_bytes = 4.0 * 4 * prob.n_unknowns
    achieved = sweep_bytes / (sweep_ms * 1e-3) / 1e9
    log("mesh3d: %d tetrahedra, %d levels (%d lagged couplings), %d iterations %.3f s: sweep %.3f ms, "
        "gradient+walls+residual %.3f ms, moments %.3f ms per iteration"
        % (prob.n_cells, prob.n_levels, prob.n_lagged, st["iters"], t, sweep_ms, st["ms_walls"] / st["iters"],
           st["ms_post"] / st["iters"]))
    out = {"metric": "cell*dir*band updates/s of steady source iterations on a tetrahedral mesh",
           "value": st["updates"] / t, "unit": "updates/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "f32 (e), f64 (gradient arithmetic, moments)", "data": "synthetic (seeded tetrahedral mesh, bands)",
           "config": {"workload": "mesh3d: 32^3 jittered cubes of a 1 um cube, six tetrahedra each, 96 directions, "
                                  "20 bands, thermalizing x walls, specular y and z walls",
                      "cells": prob.n_cells, "levels": prob.n_levels, "lagged": prob.n_lagged,
                      "iterations": st["iters"]},
           "ms_per_iteration": t / st["iters"] * 1e3,
           "phase_ms_per_iteration": {"sweep": sweep_ms, "gradient_walls_residual": st["ms_walls"] / st["iters"],
                                      "moments": st["ms_post"] / st["iters"]},
           "roofline": {"bound": "hbm", "kernel": "k_mesh_sweep_level<float> (the level launches of one sweep)",
                        "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                        "traffic": None, "avg_sweep_ms": sweep_ms, "launches_per_sweep": prob.n_levels,
                        "bytes_per_sweep": sweep_bytes}}
    print(json.dumps(out), flush=True)


def bench_tadjoint(args):
    """Transient adjoint: 500 explicit steps of the laser physics on 32^3,
    checkpoints every 50 steps, objective = weighted top-layer temperature."""
    import torch
    import bte_inputs as I
    from paper_2306_14181_amd import bte as B
    torch.cuda.set_device(0)
    cfg = I.cube3d_laser_case(n=32)
    g, mat = cfg["geometry"], cfg["material"]
    prob = B.Problem(g, mat, dict(precision=B.F32, limiter=B.LIM_NONE, dt=cfg["dt"], adjoint=True))
    P = torch.as_tensor(cfg["P"], device="cuda")
    prob.set_fields(P, torch.zeros(prob.n_cells, dtype=torch.float64, device="cuda"))
    w = torch.as_tensor(cfg["hist_weights"], device="cuda")
    n = 500
    e = prob.zeros()
    prob.transient_step(e, 5, 0.0, cfg["pulse"])
    e = prob.zeros()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob.transient_step(e, n, 0.0, cfg["pulse"])
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    t0 = time.perf_counter()
    J, grad, st = prob.transient_adjoint(prob.zeros(), n, w, 0.0, cfg["pulse"], every=50)
    torch.cuda.synchronize()
    ta = time.perf_counter() - t0
    back = st["ms_post"] / 1e3
    log("tadjoint3d: forward %d steps %.3f s, adjoint (forward + recompute + reverse) %.3f s, backward pass %.3f s"
        % (n, tf, ta, back))
    # the same adjoint with the smallest checkpoint interval that fits in
    # 90 % of the free device memory (fewer recomputed steps)
    free, _ = torch.cuda.mem_get_info()
    every_hbm = prob.transient_adjoint_interval(n, int(0.9 * free))
    hbm = None
    if every_hbm > 0:
        t0 = time.perf_counter()
        J2, grad2, st2 = prob.transient_adjoint(prob.zeros(), n, w, 0.0, cfg["pulse"], every=every_hbm)
        torch.cuda.synchronize()
        ta2 = time.perf_counter() - t0
        hbm = {"every": every_hbm, "buffer_GB": prob.transient_adjoint_bytes(n, every_hbm) / 1e9,
               "adjoint_s": ta2, "over_forward": ta2 / tf, "backward_over_forward": st2["ms_post"] / 1e3 / tf,
               "same_gradient": bool(torch.equal(grad, grad2)) and J2 == J}
        log("tadjoint3d: checkpoints every %d (%.1f GB): adjoint %.3f s, gradient identical: %s"
            % (every_hbm, hbm["buffer_GB"], ta2, hbm["same_gradient"]))
    out = {"metric": "transient adjoint cost (checkpointed reverse mode) over the forward run",
           "value": ta / tf, "unit": "ratio", "n_gpus": 1, "higher_is_better": False,
           "dtype": "f32 (e, lambda), f64 (moments, gradient)", "data": "synthetic (seeded bands, laser pulse)",
           "config": {"workload": "tadjoint3d: 32^3 cells of (2 um)^3, 128 directions, 40 bands, 500 steps, "
                                  "checkpoints every 50, limiter NONE"},
           "forward_s": tf, "adjoint_s": ta, "backward_s": back, "backward_over_forward": back / tf, "J": J,
           "forward_updates_per_s": prob.n_unknowns * n / tf, "hbm_sized_interval": hbm}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=("steady2d", "transient3d", "porous2d_batch", "porous3d_adjoint",
                                           "tadjoint3d", "ttg1d", "interface2d", "mesh2d", "mesh3d"), default="steady2d")
    ap.add_argument("--max-iter", type=int, default=1000, help="iteration cap of the converged solves")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=None,
                    help="cells per side (default: 256 for steady2d, 64 for transient3d)")
    ap.add_argument("--cg-rtol", type=float, default=1e-6)
    ap.add_argument("--cg-max-iter", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-graphs", action="store_true", help="plain launches instead of HIP graph replays")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tile shapes")
    ap.add_argument("--no-persistent", action="store_true",
                    help="2D sweeps with one launch per tile diagonal instead of one launch per sweep")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only (--gpus 1); multi-GPU sharding is not implemented",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "transient3d":
        bench_transient(args)
        return
    if args.workload == "porous2d_batch":
        bench_batch(args)
        return
    if args.workload == "porous3d_adjoint":
        bench_adjoint(args)
        return
    if args.workload == "mesh2d":
        bench_mesh(args)
        return
    if args.workload == "mesh3d":
        bench_mesh3d(args)
        return
    if args.workload == "tadjoint3d":
        bench_tadjoint(args)
        return
    if args.workload == "ttg1d":
        bench_ttg(args)
        return
    if args.workload == "interface2d":
        bench_interface(args)
        return

    import numpy as np
    import torch

    import bte_inputs as I
    from paper_2306_14181_amd import bte as B

    torch.cuda.set_device(0)
    args.n = args.n or 256
    cfg = I.square2d_source_case(n=args.n)
    geo, mat = cfg["geometry"], cfg["material"]
    P = torch.as_tensor(cfg["P"], device="cuda")
    base_ctl = dict(scheme=B.SYNTHETIC, limiter=B.LIM_NONE, cg_rtol=args.cg_rtol, cg_max_iter=args.cg_max_iter)

    results = {}
    precs = [B.F32] if args.no_fp64 else [B.F32, B.F64]
    for prec in precs:
        prob = B.Problem(geo, mat, dict(base_ctl, precision=prec))
        prob.set_graphs(not args.no_graphs)
        prob.set_persistent(not args.no_persistent)
        prob.set_fields(P, None)
        e = prob.zeros()
        tune = []
        if not args.no_autotune:
            # the sweep candidates (register tile with 2, 1, 4 rows per
            # wavefront, per-diagonal launches or one launch; LDS tiles)
            # timed on one sweep each, fastest kept
            tune = tune_sweep(B, prob, e, 3, not args.no_persistent)
            e.zero_()
        updates = prob.n_cells * prob.n_dirs * prob.n_bands
        log("precision", prec, "unknowns", prob.n_unknowns, "workspace MB %.0f" % (prob.workspace.numel() / 1e6))
        # warmup from the heat-diffusion initial guess
        tw, stw = run_steps(B, prob, e, args.warmup, True)
        log("warmup %d steps: %.3f s" % (args.warmup, tw))
        t, st = run_steps(B, prob, e, args.steps, False)
        log("timed %d steps: %.3f s  sweep %.1f ms  walls %.1f ms  post %.1f ms  cg %.1f ms (%d CG its)"
            % (args.steps, t, st["ms_sweep"], st["ms_walls"], st["ms_post"], st["ms_cg"], st["cg_iters"]))
        sweep_launch_ms = st["ms_sweep"] / max(st["sweep_launches"], 1)
        achieved = BYTES_PER_UPDATE[prec] * updates * args.steps / (st["ms_sweep"] * 1e-3) / 1e9
        # the standalone moment reduction (bte_moments: the moment kernel and
        # the per-cell finalize) over the resident state, HIP events
        prob.moments(e)
        m0, m1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        nm = 10
        m0.record()
        for _ in range(nm):
            prob.moments(e)
        m1.record()
        torch.cuda.synchronize()
        mom_ms = m0.elapsed_time(m1) / nm
        mom_GBs = BYTES_PER_UPDATE[prec] / 2 * updates / (mom_ms * 1e-3) / 1e9
        log("moments: %.3f ms per call, %.0f GB/s" % (mom_ms, mom_GBs))
        results[prec] = dict(t=t, st=st, updates=updates, achieved=achieved, prob=prob, e=e,
                             sweep_launch_ms=sweep_launch_ms, mom_ms=mom_ms, mom_GBs=mom_GBs, tune=tune)
        if args.no_accuracy:
            del prob, e
            torch.cuda.empty_cache()

    accuracy = None
    if not args.no_accuracy and B.F64 in results:
        # converge both precisions from the diffusion guess and compare
        conv = {}
        for prec, tol in ((B.F64, 1e-11), (B.F32, 1e-7)):
            r = results[prec]
            r["prob"].set_control(max_iter=3000, residual_temp=tol, residual_flux=tol * 10)
            e = r["e"]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = r["prob"].steady_solve(e, init=True, allow_not_converged=True)
            torch.cuda.synchronize()
            T, TL, q = r["prob"].moments(e)
            conv[prec] = dict(time_s=time.perf_counter() - t0, iters=st["iters"], converged=st["converged"],
                              T=T.cpu().numpy(), q=q.cpu().numpy())
            log("converge prec %d: %d iters %.2f s eps_T %.2e" % (prec, st["iters"], conv[prec]["time_s"],
                                                                 st["eps_T"]))
        T64, T32 = conv[B.F64]["T"], conv[B.F32]["T"]
        q64, q32 = conv[B.F64]["q"], conv[B.F32]["q"]
        accuracy = dict(
            T_rel_err=float(np.abs(T32 - T64).max() / np.abs(T64 - 300.0).max()),
            q_rel_err=float(np.abs(q32 - q64).max() / np.abs(q64).max()),
            iters_fp32=conv[B.F32]["iters"], iters_fp64=conv[B.F64]["iters"],
            solve_s_fp32=round(conv[B.F32]["time_s"], 3), solve_s_fp64=round(conv[B.F64]["time_s"], 3),
            reference="plain FP64 GPU run converged to eps_T 1e-11")

    r32 = results[B.F32]
    value = r32["updates"] * args.steps / r32["t"]
    launches = r32["st"]["sweep_launches"] / max(args.steps, 1)
    kept_kind = B.TUNE_SWEEP_ONE_LAUNCH if launches == 1 else B.TUNE_SWEEP
    kept = next((tuple(x["tile"]) for x in r32["tune"] if x["chosen"]), (8, 8, 2))
    kernel = ("k_sweep2d<float,NONE>, %d tile rows per wavefront" % kept[2] if kept[:2] == (8, 8)
              else "k_sweep_tile<float,2,NONE>, %dx%d LDS tiles" % kept[:2])
    out = {
        "metric": "cell*dir*band updates/s (FP32 state, FP64 moments) of steady source iterations",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r32["t"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (e), f64 (moments, CG)",
        "data": "synthetic (seeded bands, Gaussian source)",
        "config": {"workload": "square2d_source: 256x256 cells, 1 um, 20 bands, 128 directions, synthetic scheme",
                   "n": args.n, "cg_rtol": args.cg_rtol, "cg_max_iter": args.cg_max_iter},
        "roofline": {
            "bound": "hbm",
            "kernel": "%s (%s)" % (kernel, "one launch per sweep, each block waiting for its upwind tiles"
                                   if launches == 1 else "the %d tile-diagonal launches of one sweep" % launches),
            "sweep_tile": list(kept),
            "achieved": r32["achieved"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": r32["achieved"] / HBM_PEAK_GBS,
            "traffic": counter_traffic("k_sweep2d<float,0>", (kept_kind, kept)),
            "avg_launch_ms": r32["sweep_launch_ms"],
            "bytes_per_sweep": BYTES_PER_UPDATE[B.F32] * r32["updates"],
        },
        "phase_ms_per_step": {k: r32["st"][k] / args.steps for k in ("ms_sweep", "ms_walls", "ms_post", "ms_cg")},
        "autotune": [{"tile": list(x["tile"]), "kernel": x["kernel"], "ms_per_sweep": x["ms"], "chosen": x["chosen"]}
                     for x in r32["tune"]],
        "moment_reduction": {"kernel": "k_moments_band<float> + k_finalize (bte_moments)", "ms": r32["mom_ms"],
                             "achieved": r32["mom_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": r32["mom_GBs"] / HBM_PEAK_GBS, "bytes": BYTES_PER_UPDATE[B.F32] / 2 * r32["updates"]},
    }
    if B.F64 in results:
        r64 = results[B.F64]
        v64 = r64["updates"] * args.steps / r64["t"]
        out["fp64"] = {"value": v64, "ms_per_step": 1e3 * r64["t"] / args.steps,
                       "sweep_GBs": r64["achieved"], "fp32_speedup": value / v64}
    if accuracy:
        out["accuracy"] = accuracy
    if not args.no_cpu_baseline:
        for prec in list(results):
            results[prec].pop("prob", None)
            results[prec].pop("e", None)
        torch.cuda.empty_cache()
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
