#!/usr/bin/env python3
"""Benchmark of the implicit LSKUM hot path on one MI355X.

Workload: the transonic NACA 0012-type case -- 640 x 256 = 163,840-point
O-grid cloud with 4% of interior points jittered (seed 2406), Mach 0.85,
AoA 1 deg, exact-JVP modified LU-SGS in FP64, CFL 100, first-order q-derivative
pass only (no inner iterations: without a limiter the transonic start diverges
with them).
A step is one implicit iteration: q-derivatives, residual, forward and
backward colour sweeps, state update.  ``value`` is point-iterations per
second over the timed steps (HIP-graph replay, inputs resident in HBM).

Also reported: per-phase GPU times from HIP events, the roofline of the
dominant kernel, time to a 1e-8 residual drop for the exact and the
flux-difference Jacobian products, and the CPU oracle's rate on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MACH, AOA, CFL, INNER = 0.85, 1.0, 100.0, 0

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6

# Algorithmic FP64 operation count of the residual per (point, neighbour,
# split) and per (point, neighbour), with elementary functions costed at the
# operation count of a standard software evaluation (documented in the design doc).
COST = {"exp": 14, "erf": 26, "sqrt": 8, "div": 8, "log": 20}
# per neighbour: dx, dy; two q~ reconstructions (4 x 5 each); two q~ -> primitive
# conversions (11 arithmetic + exp + sqrt + 2 div each)
NB_OPS = 2 + 40 + 2 * (11 + COST["exp"] + COST["sqrt"] + 2 * COST["div"])
# per (neighbour, split): weight (3), two split fluxes (25 arithmetic + erf + exp
# + div each), difference, scale and accumulate (12)
SPLIT_OPS = 3 + 2 * (25 + COST["erf"] + COST["exp"] + COST["div"]) + 12


def residual_flops(cloud) -> float:
    """Algorithmic FP64 operations of one residual evaluation of the cloud."""
    import numpy as np
    typ = cloud.type
    deg = np.diff(cloud.nbr_off)
    active = typ != 2
    # every neighbour of an interior point lies in one x-split and one y-split
    # (ties dx == 0 / dy == 0 are rare); wall points: t-split plus n-split for
    # fluid-side neighbours, counted here as 1.5 splits per neighbour
    splits = np.where(typ == 1, 2.0, 1.5)
    return float(np.sum(deg[active] * (NB_OPS + splits[active] * SPLIT_OPS)))


def time_to_tol(lk, gc, jvp_mode, precision, max_iters):
    prm = lk.default_params(cfl=CFL, inner_iters=INNER, jvp_mode=jvp_mode, precision=precision,
                            check_every=20, tol_rel=1e-8, max_iters=max_iters)
    st = lk.State(gc, MACH, AOA, prm)
    rep = st.solve()
    out = {"converged": rep.status == 0, "iters": rep.iters, "seconds": rep.seconds,
           "res_drop": rep.res_final / rep.res_fs if rep.res_fs else None,
           "cl": rep.cl, "cd": rep.cd, "status": rep.status}
    st.close()
    return out


def cpu_baseline(cloud, iters: int):
    import oracle
    o = oracle.Oracle(cloud, mach=MACH, aoa_deg=AOA, cfl=CFL, inner_iters=INNER)
    U = o.free_stream()
    t0 = time.perf_counter()
    for _ in range(iters):
        U, _, _, _ = o.iteration(U)
    dt = time.perf_counter() - t0
    return {"value": cloud.n * iters / dt, "unit": "point-iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} serial FP64 oracle iterations of the {cloud.n}-point workload "
                      f"from the free-stream start ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--tol-iters", type=int, default=20000,
                    help="iteration cap of the time-to-1e-8 runs (0 skips them)")
    ap.add_argument("--cpu-iters", type=int, default=4, help="oracle iterations (0 skips)")
    ap.add_argument("--profile-only", action="store_true",
                    help="run only the timed steps (for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path "
              "(see DESIGN.md for how it would shard)", file=sys.stderr)
        sys.exit(2)
    if args.steps % 10 or args.warmup % 10:
        print("--steps and --warmup must be multiples of 10", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2406_07441_amd import cloudgen
    from paper_2406_07441_amd import lskum as lk

    torch.cuda.set_device(0)
    cloud = cloudgen.cloud_163840()
    gc = lk.Cloud(cloud)
    prm = lk.default_params(cfl=CFL, inner_iters=INNER, check_every=10, tol_rel=0.0,
                            max_iters=args.warmup)
    st = lk.State(gc, MACH, AOA, prm)
    print(f"# cloud n={cloud.n} nnz={cloud.nnz} colours={gc.n_colours} "
          f"degenerate={gc.n_degenerate}", file=sys.stderr, flush=True)
    st.solve()                                    # warmup (captures the graph)
    prm.max_iters = args.steps
    st.set_params(prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = st.solve()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if rep.iters != args.steps:
        print(f"timed solve stopped after {rep.iters} steps (status {rep.status})",
              file=sys.stderr)
        sys.exit(1)
    value = cloud.n * args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    print(f"# timed {args.steps} steps: {ms_per_step:.4f} ms/step, res {rep.res_final:.3e}",
          file=sys.stderr, flush=True)

    # per-phase GPU times (HIP events on the library's stream)
    nt = 20
    acc = None
    for _ in range(nt):
        ph = st.step_timed()
        acc = ph if acc is None else {k: acc[k] + ph[k] for k in acc}
    phases = {k: v / nt for k, v in acc.items()}
    res_ms = phases["residual"]
    flops = residual_flops(cloud)
    achieved = flops / (res_ms * 1e-3) / 1e12
    roofline = {"kernel": "k_residual", "bound": "alu", "achieved": achieved,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                "traffic": None, "flops_per_launch": flops, "avg_ms": res_ms}
    st.close()
    if args.profile_only:
        print(json.dumps({"ms_per_step": ms_per_step, "phases_ms": phases}))
        return

    extra = {}
    if args.tol_iters > 0:
        extra["time_to_1e-8"] = {
            "exact_fp64": time_to_tol(lk, gc, lk.JVP_EXACT, lk.FP64, args.tol_iters),
            "fluxdiff_fp64": time_to_tol(lk, gc, lk.JVP_FLUXDIFF, lk.FP64, args.tol_iters),
            "exact_mixed": time_to_tol(lk, gc, lk.JVP_EXACT, lk.MIXED, args.tol_iters),
        }
        print(f"# time to tol: {json.dumps(extra['time_to_1e-8'])}", file=sys.stderr, flush=True)
    cpu = cpu_baseline(cloud, args.cpu_iters) if args.cpu_iters > 0 else None

    line = {
        "metric": "point-iters/s + time to 1e-8 res drop: exact-JVP LU-SGS FP64 vs mixed+batched",
        "value": value, "unit": "point-iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "O-grid NACA0012-type cloud 640x256=163840 pts, 4% jittered, "
                               "M0.85 AoA1, exact-JVP LU-SGS FP64, CFL100, no inner iterations",
                   "points": cloud.n, "edges": cloud.nnz, "colours": gc.n_colours},
        "roofline": roofline, "cpu_baseline": cpu, "phases_ms": phases, **extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
