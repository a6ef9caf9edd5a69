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

Prints one JSON line.  --gpus N > 1 is not supported on this build.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
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


def cpu_baseline(cfg, seconds_hint=30.0):
    """Oracle (FP64 C, OpenMP) on a bounded sample: one source iteration of the
    same workload (sweep, moments, synthetic correction), started from the
    heat-diffusion state (computed untimed)."""
    import numpy as np
    import oracle as O
    case = O.Case(cfg["geometry"], cfg["material"], P=cfg["P"])
    Td = O.diffusion_T(case, rtol=1e-10)
    e0 = (case.C[None, None, :] * Td[:, None, None] / (4 * np.pi) * np.ones((1, case.na, 1))).reshape(-1)
    del Td
    t0 = time.perf_counter()
    e1, st = O.steady(case, scheme=1, tol_T=0.0, tol_q=0.0, max_iter=1, cg_rtol=1e-6, e=e0)
    dt = time.perf_counter() - t0
    updates = case.nc * case.na * case.nl
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=updates / dt, unit="cell*dir*band updates/s", cores=threads, kind="oracle",
                sample="1 source iteration (sweep + FP64 moments + CG correction) of the 256x256 x 128 dir x "
                       "20 band workload, %.1f s" % dt)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256, help="cells per side (256 = the benchmark workload)")
    ap.add_argument("--cg-rtol", type=float, default=1e-6)
    ap.add_argument("--cg-max-iter", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (--gpus 1); multi-GPU sharding is not implemented",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import bte_inputs as I
    from paper_2306_14181_amd import bte as B

    torch.cuda.set_device(0)
    cfg = I.config1(n=args.n)
    geo, mat = cfg["geometry"], cfg["material"]
    P = torch.as_tensor(cfg["P"], device="cuda")
    base_ctl = dict(scheme=B.SYNTHETIC, limiter=B.LIM_NONE, cg_rtol=args.cg_rtol, cg_max_iter=args.cg_max_iter)

    results = {}
    precs = [B.F32] if args.no_fp64 else [B.F32, B.F64]
    for prec in precs:
        prob = B.Problem(geo, mat, dict(base_ctl, precision=prec))
        prob.set_fields(P, None)
        e = prob.zeros()
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
        results[prec] = dict(t=t, st=st, updates=updates, achieved=achieved, prob=prob, e=e,
                             sweep_launch_ms=sweep_launch_ms)
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
            "kernel": "k_sweep<float> (all tile-wavefront launches of one sweep)",
            "achieved": r32["achieved"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": r32["achieved"] / HBM_PEAK_GBS,
            "traffic": None,
            "avg_launch_ms": r32["sweep_launch_ms"],
        },
        "phase_ms_per_step": {k: r32["st"][k] / args.steps for k in ("ms_sweep", "ms_walls", "ms_post", "ms_cg")},
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
