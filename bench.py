"""Benchmark of the implicit LSKUM hot path on one MI355X.

Workload (the timed steps): a 2560 x 1024 = 2,621,440-point O-grid cloud
around the 12%-thick symmetric profile (first normal spacing equal to the mean
wall spacing), Mach 0.5, AoA 3 deg; exact-JVP modified LU-SGS in FP64, CFL 100,
one inner iteration of the q-derivatives and the Venkatakrishnan limiter (K 5)
on the q~ reconstruction (the impulsive free-stream start goes non-physical on
this cloud without it; the paper names no limiter).  A step is one implicit
iteration: q-derivatives, limiter, residual with the local time step, diagonal
and linearisation data, residual norm, forward and backward colour sweeps,
state update.  ``value`` is point-iterations per second over the timed steps
(HIP-graph replay, every array resident in HBM).

Also reported: per-phase GPU times from HIP events, the roofline of every
kernel against the algorithmic work per point, the same workload in mixed
precision, time to a 1e-8 residual drop on the 163,840-point transonic cloud
with exact and flux-difference Jacobian products (FP64) and mixed precision,
the explicit solver beside the implicit one, the batched 64-condition
workload, the learned warm start, and the CPU oracle's rate on a bounded
sample of the timed workload (all host cores).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# the timed workload
HEAD_MACH, HEAD_AOA = 0.5, 3.0
# the transonic 163,840-point workload of the time-to-tolerance legs
MACH, AOA = 0.85, 1.0
CFL, INNER, LIMITER, LIMITER_K = 100.0, 1, 1, 5.0

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz

# Algorithmic FP64 operation count of the residual, with elementary functions
# costed at the operation count of a standard software evaluation.
COST = {"exp": 14, "erf": 26, "sqrt": 8, "div": 8, "log": 20}
# per neighbour: dx, dy; two q~ reconstructions (4 x 5 each); two q~ -> primitive
# conversions (11 arithmetic + exp + sqrt + 2 div each)
NB_OPS = 2 + 40 + 2 * (11 + COST["exp"] + COST["sqrt"] + 2 * COST["div"])
# per (neighbour, split): weight (3), two split fluxes (25 arithmetic + erf + exp
# + div each), difference, scale and accumulate (12)
SPLIT_OPS = 3 + 2 * (25 + COST["erf"] + COST["exp"] + COST["div"]) + 12

# Algorithmic HBM bytes per point of each phase: every array read or written
# once, neighbour data reused from cache, an interior point's 24-entry stencil
# (CSR about 100 bytes); FP64.
QGRAD_FIRST_B = 244   # U 32, xy 16, CSR 100 -> q, q_x, q_y 96
QGRAD_INNER_B = 276   # q, q_x, q_y 96, xy 16, CSR 100 -> q_x, q_y 64
LIMITER_B = 64        # the limited q_x, q_y written by the last pass (the limiter is an addition)
RESIDUAL_B = 390      # q, q_x, q_y 96, xy 16, CSR 100, U 32 -> R 32, D and dt 16, linearisation 96
NORM_B = 8            # R_rho^2
SWEEP_FWD_B = 320     # R 32, D 8, CSR 100, xy 16, neighbours' linearisation 96, dU* 32 -> dU* 32
SWEEP_BWD_B = 284     # dU* 32, D 8, CSR 100, xy 16, neighbours' linearisation 96 -> dU 32
UPDATE_B = 128        # U 32, dU 32 -> U 32, q 32


def residual_flops(cloud) -> float:
    """Algorithmic FP64 operations of one residual evaluation of the cloud."""
    import numpy as np
    typ = cloud.type
    deg = np.diff(cloud.nbr_off)
    active = typ != 2
    # every neighbour of an interior point lies in one x-split and one y-split;
    # wall points: t-split plus the n-split for fluid-side neighbours (1.5)
    splits = np.where(typ == 1, 2.0, 1.5)
    return float(np.sum(deg[active] * (NB_OPS + splits[active] * SPLIT_OPS)))


def sweep_points(colours) -> tuple[int, int, int]:
    """Points swept by the forward colour-phase launches (colours 1 and up: the
    colour-0 phase has no lower neighbours and is formed inside the residual
    kernel), by the backward launches (all but the top colour, whose backward
    phase is the identity), and the number of launches per direction."""
    import numpy as np
    top = int(colours.max())
    return (int(np.count_nonzero(colours > 0)), int(np.count_nonzero(colours < top)), top)


def iteration_bytes(n: int, inner: int = INNER, limiter: bool = True) -> float:
    """Algorithmic HBM bytes of one whole iteration of n points."""
    per_point = (QGRAD_FIRST_B + inner * QGRAD_INNER_B + (LIMITER_B if limiter else 0)
                 + RESIDUAL_B + NORM_B + SWEEP_FWD_B + SWEEP_BWD_B + UPDATE_B)
    return float(n * per_point)


def kernel_rooflines(cloud, colours, phases: dict) -> dict:
    """Roofline of each kernel of a step from its HIP-event phase time:
    algorithmic work per launch / average launch duration."""
    n = cloud.n
    fwd_pts, bwd_pts, launches = sweep_points(colours)
    flops = residual_flops(cloud)

    def hbm(b_per_step, ms, nl):
        gbs = b_per_step / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": gbs / PEAK_HBM_GBS, "bytes_per_launch": b_per_step / nl,
                "avg_ms": ms / nl, "launches_per_step": nl, "ms_per_step": ms}

    tf = flops / (phases["residual"] * 1e-3) / 1e12
    out = {
        "k_residual": {"bound": "alu", "achieved": tf, "peak": PEAK_FP64_TFLOPS,
                       "unit": "TFLOP/s", "frac": tf / PEAK_FP64_TFLOPS,
                       "flops_per_launch": flops, "avg_ms": phases["residual"],
                       "launches_per_step": 1, "ms_per_step": phases["residual"],
                       "bytes_per_launch": float(n * RESIDUAL_B)},
        "k_sweep forward": hbm(fwd_pts * SWEEP_FWD_B, phases["forward_sweep"], launches),
        "k_sweep backward": hbm(bwd_pts * SWEEP_BWD_B, phases["backward_sweep"], launches),
        "k_qgrad (both passes)": hbm(n * (QGRAD_FIRST_B + INNER * QGRAD_INNER_B + LIMITER_B),
                                     phases["q_derivatives"], 1 + INNER),
        "k_update": hbm(n * UPDATE_B, phases["update"], 1),
        "k_norm_partial + k_norm_comp": hbm(n * NORM_B, phases["norm"], 2),
    }
    return out


def device_source_hash() -> str:
    """The library's build hash: its sources, headers and compiler flags."""
    from paper_2406_07441_amd import build
    return build.source_hash()


TRAFFIC_FILE = {"fp64": "traffic_2621440_fp64.md", "mixed": "traffic_2621440_mixed.md"}


def measured_traffic(precision: str = "fp64"):
    """HBM bytes per launch of each kernel of the timed workload from rocprofv3
    FETCH_SIZE/WRITE_SIZE counter runs, when the summary in profiles/ was taken
    on the current kernel source."""
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILE[precision])
    if not os.path.exists(path):
        return None
    out = {}
    for line in open(path):
        if line.startswith("source_sha256:"):
            if line.split(":", 1)[1].strip() != device_source_hash():
                return None
        if line.startswith("| `") and "|" in line[3:]:
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            try:
                out[cells[0].strip("`")] = float(cells[-1])
            except ValueError:
                pass
    return out or None


def params(lk, **kw):
    base = dict(cfl=CFL, inner_iters=INNER, limiter=LIMITER, limiter_k=LIMITER_K)
    base.update(kw)
    return lk.default_params(**base)


def time_to_tol(lk, gc, max_iters, **kw):
    prm = params(lk, check_every=100, tol_rel=1e-8, max_iters=max_iters, **kw)
    st = lk.State(gc, MACH, AOA, prm)
    rep = st.solve()
    out = {"converged": rep.status == 0, "iters": rep.iters, "seconds": rep.seconds,
           "res_drop": rep.res_final / rep.res_fs if rep.res_fs else None,
           "cl": rep.cl, "cd": rep.cd}
    st.close()
    return out


def explicit_vs_implicit(lk, gc, iters):
    """The paper's explicit solver (U - dt R, CFL 0.4) against the implicit one
    (CFL 100) on the benchmark workload: time per iteration and residual drop
    after the same number of iterations."""
    out = {}
    for name, kw in (("implicit_fp64", dict()), ("explicit_fp64", dict(scheme=lk.EXPLICIT,
                                                                        cfl=0.4))):
        prm = params(lk, check_every=100, tol_rel=0.0, max_iters=iters, **kw)
        st = lk.State(gc, MACH, AOA, prm)
        rep = st.solve()
        out[name] = {"iters": rep.iters, "status": rep.status, "seconds": rep.seconds,
                     "ms_per_iter": 1e3 * rep.seconds / max(1, rep.iters),
                     "res_drop": rep.res_final / rep.res_fs}
        st.close()
    return out


def residual_histories(lk, cloudgen, max_iters=20000, chunk=200):
    """The 160 x 40 cloud (M 0.63, 2 deg, no limiter: the paper's scheme as
    written) solved to 1e-8 with exact tangents and with flux differences in
    FP64: iterations, time and the residual drop every `chunk` iterations --
    the convergence-rate comparison of the paper's residual histories."""
    cloud = cloudgen.cloud_6400()
    gc = lk.Cloud(cloud)
    out = {"workload": "O-grid 160x40=6400 pts, M0.63 AoA2, CFL100, m=1, no limiter"}
    for name, mode in (("exact", lk.JVP_EXACT), ("fluxdiff", lk.JVP_FLUXDIFF)):
        prm = lk.default_params(cfl=CFL, inner_iters=INNER, jvp_mode=mode, check_every=chunk,
                                tol_rel=1e-8, max_iters=chunk)
        st = lk.State(gc, 0.63, 2.0, prm)
        hist, it, secs, status = [], 0, 0.0, -6
        while it < max_iters:
            rep = st.solve()
            it += rep.iters
            secs += rep.seconds
            hist.append(float(f"{rep.res_final / rep.res_fs:.4e}"))
            if rep.status != -6:
                status = rep.status
                break
        cl, cd = st.forces()
        out[name] = {"iters": it, "status": status, "seconds": secs, "cl": cl, "cd": cd,
                     f"res_drop_every_{chunk}": hist}
        st.close()
    gc.close()
    return out


def batch_run(lk, cloudgen, iters):
    """64 conditions on 8 uneven clouds, FP32 sweeps / FP64 residual, autotuned."""
    import numpy as np
    clouds = cloudgen.batch_clouds()
    gcs = [lk.Cloud(c) for c in clouds]
    mach, aoa = cloudgen.batch_conditions()
    prm = lk.default_params(cfl=CFL, inner_iters=INNER, precision=lk.MIXED, limiter=LIMITER,
                            limiter_k=LIMITER_K, check_every=50, tol_rel=0.0, max_iters=iters)
    b = lk.Batch(gcs, np.arange(64) % 8, mach, aoa, prm)
    lanes = b.autotune(2)
    reps, tot = b.solve()
    pts = sum(r["iters"] * b.sizes[k] for k, r in enumerate(reps))
    # algorithmic bytes: each condition's iterations on its own cloud
    moved = sum(iteration_bytes(r["iters"] * b.sizes[k]) for k, r in enumerate(reps))
    out = {"conditions": 64, "clouds": [c.n for c in clouds], "points": b.n_points,
           "colour_phases": b.n_colours, "iters": iters, "seconds": tot,
           "point_iters_per_s": pts / tot, "iteration_gbs": moved / tot / 1e9,
           "iteration_frac_hbm": moved / tot / 1e9 / PEAK_HBM_GBS,
           "lanes": {"sweep": lanes[0], "residual": lanes[1], "qgrad": lanes[2]},
           "failed": int(sum(r["status"] == lk.ERR_NONPHYSICAL for r in reps)),
           "median_res_drop": float(np.median([r["res_final"] / r["res_fs"] for r in reps]))}
    b.close()
    return out


CHUNK_ITERS = 2000   # long solves run in chunks, each printing a progress line


def solve_chunked(obj, prm, max_iters, n_cond, label, max_seconds=0.0):
    """Solves a State (n_cond 1) or Batch to its tolerance in chunks of
    CHUNK_ITERS iterations; returns per-condition (iters, seconds, status, cl,
    cd) at first convergence and the total seconds.  max_seconds > 0 stops
    after the chunk that passes it."""
    done = [None] * n_cond
    total_it, total_s = 0, 0.0
    last = None
    while total_it < max_iters and any(d is None for d in done):
        if max_seconds > 0 and total_s >= max_seconds:
            break
        prm.max_iters = min(CHUNK_ITERS, max_iters - total_it)
        obj.set_params(prm)
        if n_cond == 1:
            r = obj.solve()
            reps, secs = [r.as_dict()], r.seconds
        else:
            reps, secs = obj.solve()
        for k, r in enumerate(reps):
            if done[k] is None and r["status"] == 0:
                done[k] = {"iters": total_it + r["iters"], "seconds": total_s + r["seconds"],
                           "status": 0, "cl": r["cl"], "cd": r["cd"], "res_fs": r["res_fs"],
                           "res_drop": r["res_final"] / r["res_fs"]}
        total_it += prm.max_iters
        total_s += secs
        last = reps
        print(f"# {label}: {total_it} iterations, {total_s:.1f} s, "
              f"{sum(d is not None for d in done)}/{n_cond} converged", file=sys.stderr, flush=True)
        if any(r["status"] == -5 for r in reps):
            break
    for k in range(n_cond):
        if done[k] is None:
            done[k] = {"iters": total_it, "seconds": total_s, "status": last[k]["status"],
                       "cl": last[k]["cl"], "cd": last[k]["cd"], "res_fs": last[k]["res_fs"],
                       "res_drop": last[k]["res_final"] / last[k]["res_fs"]}
    return done, total_s


# Residual-driven CFL control of the batch (a reading of our own: the paper
# runs one CFL number): a condition whose residual reaches no new minimum over
# a window of iterations has its CFL number cut by a factor, down to a floor.
CFL_WINDOW, CFL_FACTOR, CFL_MIN = 2000, 0.3, 9.0


def batch_converge(lk, cloudgen, max_iters, max_seconds=0.0):
    """The 64-condition batch solved to 1e-8 of each condition's free-stream
    residual with the per-condition CFL control: time until all retire,
    per-condition iterations and final CFL numbers.  max_seconds > 0 stops
    after the chunk that passes it (the rest are listed as not converged)."""
    import numpy as np
    clouds = cloudgen.batch_clouds()
    gcs = [lk.Cloud(c) for c in clouds]
    mach, aoa = cloudgen.batch_conditions()
    prm = lk.default_params(cfl=CFL, inner_iters=INNER, precision=lk.MIXED, limiter=LIMITER,
                            limiter_k=LIMITER_K, check_every=100, tol_rel=1e-8)
    b = lk.Batch(gcs, np.arange(64) % 8, mach, aoa, prm)
    lanes = b.autotune(2)
    prm.sweep_lanes, prm.residual_lanes, prm.qgrad_lanes = lanes
    b.set_cfl_control(CFL_WINDOW, CFL_FACTOR, CFL_MIN)
    done, tot = solve_chunked(b, prm, max_iters, 64, "batch to 1e-8", max_seconds)
    pts = sum(d["iters"] * b.sizes[k] for k, d in enumerate(done))
    conv = [d["seconds"] for d in done if d["status"] == 0]
    out = {"conditions": 64, "points": b.n_points,
           "cfl_control": {"window": CFL_WINDOW, "factor": CFL_FACTOR, "cfl_min": CFL_MIN},
           "seconds_until_all_retired": max(conv) if len(conv) == 64 else None,
           "seconds_run": tot, "converged": len(conv),
           "point_iters_per_s": pts / tot,
           "lanes": {"sweep": lanes[0], "residual": lanes[1], "qgrad": lanes[2]},
           "iters": [d["iters"] for d in done],
           "final_cfl": [float(f"{c:.3g}") for c in b.get_cfl()],
           "res_drop": [float(f"{d['res_drop']:.3e}") for d in done],
           "not_converged": [k for k, d in enumerate(done) if d["status"] != 0]}
    b.close()
    return out


def config3_run(lk, cloudgen, max_iters, precisions=("fp64", "mixed")):
    """2560 x 1024 cloud, M 0.5, AoA 3 deg: FP64 against mixed precision to 1e-8
    (limiter on: without it the impulsive start goes non-physical on this cloud
    within 2,000 iterations)."""
    import numpy as np
    cloud = cloudgen.cloud_2621440()
    gc = lk.Cloud(cloud)
    out, U = {}, {}
    for name, prec in (("fp64", lk.FP64), ("mixed", lk.MIXED)):
        if name not in precisions:
            continue
        prm = lk.default_params(cfl=CFL, inner_iters=INNER, precision=prec, check_every=100,
                                tol_rel=1e-8, limiter=LIMITER, limiter_k=LIMITER_K)
        st = lk.State(gc, 0.5, 3.0, prm)
        (d,), secs = solve_chunked(st, prm, max_iters, 1, f"2.6M {name}")
        U[name] = st.get_U()
        out[name] = {"converged": d["status"] == 0, "iters": d["iters"], "seconds": d["seconds"],
                     "point_iters_per_s": cloud.n * d["iters"] / d["seconds"],
                     "res_drop": d["res_drop"], "cl": d["cl"], "cd": d["cd"]}
        st.close()
    if len(U) == 2:
        out["max_abs_dU_mixed_vs_fp64"] = float(np.abs(U["mixed"] - U["fp64"]).max())
        out["dcl"] = out["mixed"]["cl"] - out["fp64"]["cl"]
        out["dcd"] = out["mixed"]["cd"] - out["fp64"]["cd"]
    out["points"] = cloud.n
    return out


MLP_FLOP_PER_ROW = 2 * (5 * 128 + 2 * 128 * 128 + 128 * 4)   # 67,840
PEAK_BF16_TFLOPS = 2500.0


# Warm-start leg sizes, scaled down from the recipe's 512 training fields and 32
# held-out conditions on a 640,000-point cloud to fit a benchmark job:
# (training conditions, training clouds, their size range, held-out cloud).
WARM_SCALES = {
    "default": (32, 4, 20_000, 60_000, (640, 256)),
    "large": (64, 8, 40_000, 80_000, (1280, 500)),
    "xlarge": (128, 16, 40_000, 80_000, (1280, 500)),
}


def warm_start_run(lk, cloudgen, train_steps: int, held_out: int, scale: str = "default"):
    """Learned warm start, scaled down from the 640k-point / 512-field recipe
    (WARM_SCALES): converged fields of the training conditions on small clouds
    (the batched solver in mixed precision, to 1e-6) train the network;
    `held_out` conditions on a held-out cloud are then solved to 1e-8 of each
    condition's free-stream residual three ways: the plain FP64 solver one
    condition at a time from the free stream (baseline); the mixed-precision
    batch from the free stream; the mixed-precision batch from the warm start."""
    import numpy as np
    import torch
    n_train, n_clouds, nmin, nmax, (hw, hk) = WARM_SCALES[scale]
    clouds = cloudgen.batch_clouds(seed=40, count=n_clouds, nmin=nmin, nmax=nmax)
    gcs = [lk.Cloud(c) for c in clouds]
    mach, aoa = cloudgen.batch_conditions(seed=41, count=n_train)
    prm = lk.default_params(cfl=CFL, inner_iters=INNER, precision=lk.MIXED, limiter=LIMITER,
                            limiter_k=LIMITER_K, check_every=50, tol_rel=1e-6, max_iters=40000)
    t0 = time.perf_counter()
    b = lk.Batch(gcs, np.arange(n_train) % n_clouds, mach, aoa, prm)
    reps, _ = b.solve()
    ok = [r["status"] == 0 for r in reps]
    X, T = b.features(targets=True)
    # rows of conditions that did not converge are left out of the training set
    keep = torch.cat([torch.full((b.sizes[k],), bool(ok[k]), device="cuda")
                      for k in range(n_train)])
    X, T = X[keep].contiguous(), T[keep].contiguous()
    b.close()
    gen_s = time.perf_counter() - t0
    print(f"# warm start: {int(sum(ok))}/{n_train} training fields in {gen_s:.1f} s",
          file=sys.stderr, flush=True)
    net = lk.MLP(seed=11, max_rows=8192)
    hist, train_s = net.train(X, T, steps=train_steps, batch=8192, lr=3e-3, lr_final=1e-5, seed=13)
    rows = X.shape[0]
    print(f"# warm start: trained {train_steps} steps in {train_s:.1f} s", file=sys.stderr,
          flush=True)

    held = cloudgen.ogrid(hw, hk, r=None, t=0.12, name=f"heldout{hw}x{hk}")
    gh = lk.Cloud(held)
    hm, ha = cloudgen.batch_conditions(seed=42, count=held_out)
    common = dict(cfl=CFL, inner_iters=INNER, limiter=LIMITER, limiter_k=LIMITER_K,
                  check_every=50, tol_rel=1e-8, max_iters=150000)
    # (a) baseline: plain FP64 solver, one condition at a time, free-stream start
    base = []
    for m, a_ in zip(hm, ha):
        st = lk.State(gh, float(m), float(a_), lk.default_params(**common))
        r = st.solve()
        base.append(r.as_dict())
        st.close()
        print(f"# warm start: FP64 baseline M {float(m):.3f} AoA {float(a_):.2f}: {r.iters} "
              f"iterations, {r.seconds:.1f} s", file=sys.stderr, flush=True)
    base_s = sum(r["seconds"] for r in base)
    print(f"# warm start: FP64 baseline {base_s:.1f} s", file=sys.stderr, flush=True)
    cc = np.zeros(held_out, np.int32)
    prm_mx = lk.default_params(precision=lk.MIXED, **common)
    # (b) mixed-precision batch, free-stream start
    bf = lk.Batch([gh], cc, hm, ha, prm_mx)
    r_bf, t_bf = solve_chunked(bf, prm_mx, common["max_iters"], held_out, "held-out mixed batch")
    bf.close()
    print(f"# warm start: mixed batch from the free stream {t_bf:.1f} s", file=sys.stderr,
          flush=True)
    # (c) mixed-precision batch, warm start (inference and residual check inside the timing)
    bw = lk.Batch([gh], cc, hm, ha, prm_mx)
    Xh = bw.features()
    net.forward(Xh)   # the first call loads the kernel; the timing takes the next five
    torch.cuda.synchronize()
    ti = time.perf_counter()
    for _ in range(5):
        net.forward(Xh)
    torch.cuda.synchronize()
    infer_s = (time.perf_counter() - ti) / 5
    tw = time.perf_counter()
    fb, res_w = net.warm_start(bw)
    warm_s = time.perf_counter() - tw
    r_bw, t_bw = solve_chunked(bw, prm_mx, common["max_iters"], held_out,
                               "held-out warm-started batch")
    bw.close()
    net.close()
    return {
        "scale": scale,
        "training": {"clouds": [c.n for c in clouds], "conditions": n_train,
                     "converged": int(sum(ok)), "rows": rows, "field_gen_s": gen_s,
                     "steps": train_steps, "batch": 8192, "train_s": train_s,
                     "loss_first": float(hist[:10].mean()), "loss_last": float(hist[-50:].mean()),
                     "train_tflops": 3 * MLP_FLOP_PER_ROW * 8192 * train_steps / train_s / 1e12},
        "held_out": {
            "cloud": held.n, "conditions": [[float(m), float(a_)] for m, a_ in zip(hm, ha)],
            "fp64_single_free_stream": {"iters": [r["iters"] for r in base],
                                        "status": [r["status"] for r in base],
                                        "seconds": base_s},
            "mixed_batch_free_stream": {"iters": [r["iters"] for r in r_bf],
                                        "status": [r["status"] for r in r_bf],
                                        "seconds": t_bf},
            "mixed_batch_warm_start": {"iters": [r["iters"] for r in r_bw],
                                       "status": [r["status"] for r in r_bw],
                                       "seconds": t_bw + warm_s, "warm_start_s": warm_s,
                                       "fallback": fb.tolist(),
                                       "res_warm_over_res_fs": [float(res_w[k] / r_bw[k]["res_fs"])
                                                                for k in range(held_out)]},
            "speedup_vs_fp64_baseline": base_s / (t_bw + warm_s),
            "warm_start_iteration_saving": 1.0 - sum(r["iters"] for r in r_bw)
            / max(1, sum(r["iters"] for r in r_bf)),
            "max_abs_dcl_vs_baseline": max(abs(r_bw[k]["cl"] - base[k]["cl"])
                                           for k in range(held_out)),
            "max_abs_dcd_vs_baseline": max(abs(r_bw[k]["cd"] - base[k]["cd"])
                                           for k in range(held_out))},
        "inference": {"rows": int(Xh.shape[0]), "seconds": infer_s,
                      "tflops": MLP_FLOP_PER_ROW * Xh.shape[0] / infer_s / 1e12,
                      "frac_bf16_peak": MLP_FLOP_PER_ROW * Xh.shape[0] / infer_s / 1e12
                      / PEAK_BF16_TFLOPS},
    }


def mlp_profile_run(lk) -> dict:
    """The warm-start network alone on random rows: 20 + 200 minibatch Adam
    steps of 8192 rows, then 11 forward passes over 655,360 rows and 11 over
    1,000,000 rows (one launch each)."""
    import numpy as np
    import torch
    rng = np.random.default_rng(0)
    n = 1_000_000
    X = torch.from_numpy(rng.uniform(-1, 1, (n, 5)).astype(np.float32)).cuda()
    T = torch.from_numpy((0.1 * rng.standard_normal((n, 4))).astype(np.float32)).cuda()
    net = lk.MLP(seed=1, max_rows=8192)
    net.train(X, T, steps=20, batch=8192, lr=1e-3)
    _, train_s = net.train(X, T, steps=200, batch=8192, lr=1e-3)
    out = {"train_steps": 200, "batch": 8192, "train_s": train_s,
           "train_tflops": 3 * MLP_FLOP_PER_ROW * 8192 * 200 / train_s / 1e12}
    net.close()
    big = lk.MLP(seed=1, max_rows=n)
    for rows in (655_360, n):
        big.forward(X[:rows])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            big.forward(X[:rows])
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 10
        out[f"forward_{rows}_ms"] = 1e3 * dt
        out[f"forward_{rows}_tflops"] = MLP_FLOP_PER_ROW * rows / dt / 1e12
    big.close()
    return out


def cpu_baseline(cloud, mach, aoa, min_seconds: float = 10.0, max_iters: int = 8):
    """The CPU oracle (serial arithmetic, per-point loops and the points of a
    colour over OpenMP threads, results independent of the thread count) on
    the timed workload: whole iterations from the free-stream start until
    min_seconds have passed or max_iters iterations have run."""
    import oracle
    o = oracle.Oracle(cloud, mach=mach, aoa_deg=aoa, cfl=CFL, inner_iters=INNER,
                      limiter=LIMITER, limiter_k=LIMITER_K)
    U = o.free_stream()
    t0 = time.perf_counter()
    it = 0
    while it < max_iters and (it == 0 or time.perf_counter() - t0 < min_seconds):
        U, _, _, _ = o.iteration(U)
        it += 1
    dt = time.perf_counter() - t0
    cores = oracle.threads()
    return {"value": cloud.n * it / dt, "unit": "point-iters/s", "cores": cores, "kind": "oracle",
            "sample": f"{it} FP64 oracle iterations of the timed {cloud.n}-point workload from "
                      f"the free-stream start ({dt:.1f} s), {cores} OpenMP threads on "
                      f"{host_cpu()}"}


def host_cpu() -> str:
    """The host processor model and its logical CPU count."""
    model = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return f"{model} ({os.cpu_count()} logical CPUs)"


def check_every_for(steps: int) -> int:
    """Iterations per captured graph: the largest of 40, 20, 10, 5, 4, 2, 1
    that divides the timed step count (the library runs any remainder
    eagerly, so this only sets how often the host reads the residual)."""
    for d in (40, 20, 10, 5, 4, 2, 1):
        if steps % d == 0:
            return d
    return 1


def timed_run(lk, gc, mach, aoa, steps: int, warmup: int, precision, label: str):
    """`warmup` untimed steps (the first captures the iteration graph), then
    `steps` timed graph-replayed steps; then 10 eager steps with HIP events
    between the phases.  Returns (seconds, report, phase ms)."""
    import torch
    every = check_every_for(steps)
    prm = params(lk, check_every=every, tol_rel=0.0, max_iters=warmup, precision=precision)
    st = lk.State(gc, mach, aoa, prm)
    st.solve()   # captures the graph even for warmup == 0
    prm.max_iters = steps
    st.set_params(prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = st.solve()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if rep.iters != steps:
        st.close()
        raise RuntimeError(f"{label}: timed solve stopped after {rep.iters} of {steps} steps "
                           f"(status {rep.status})")
    nt = 10
    acc = None
    for _ in range(nt):
        ph = st.step_timed()
        acc = ph if acc is None else {k: acc[k] + ph[k] for k in acc}
    phases = {k: v / nt for k, v in acc.items()}
    st.close()
    print(f"# {label}: {steps} steps in {elapsed:.4f} s ({1e3 * elapsed / max(1, steps):.4f} "
          f"ms/step), res {rep.res_final:.3e}; phases {json.dumps(phases)}",
          file=sys.stderr, flush=True)
    return elapsed, rep, phases


def parse_args(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision run of the timed workload")
    ap.add_argument("--tol-iters", type=int, default=60000,
                    help="iteration cap of the 163,840-point time-to-1e-8 runs (0 skips them)")
    ap.add_argument("--batch-iters", type=int, default=100,
                    help="iterations of the 64-condition batch run (0 skips it)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum duration of the oracle sample (0 skips it)")
    ap.add_argument("--warm-steps", type=int, default=6000,
                    help="training steps of the warm-start leg (0 skips it)")
    ap.add_argument("--warm-held-out", type=int, default=4,
                    help="held-out conditions of the warm-start leg")
    ap.add_argument("--warm-scale", default="default", choices=sorted(WARM_SCALES),
                    help="training and held-out sizes of the warm-start leg")
    ap.add_argument("--batch-converge-iters", type=int, default=0,
                    help="solve the 64-condition batch to 1e-8 with this cap (0 skips)")
    ap.add_argument("--batch-converge-seconds", type=float, default=0.0,
                    help="stop the batch-to-1e-8 leg after this many seconds (0: no limit)")
    ap.add_argument("--histories", action="store_true",
                    help="residual histories to 1e-8 on the 6,400-point cloud, exact vs "
                         "flux-difference products")
    ap.add_argument("--config3-iters", type=int, default=0,
                    help="2,621,440-point FP64 vs mixed run to 1e-8 with this cap (0 skips)")
    ap.add_argument("--config3-precisions", default="fp64,mixed",
                    help="precisions of the --config3-iters leg (comma separated)")
    ap.add_argument("--profile-only", action="store_true",
                    help="run only the timed steps (for profiler runs)")
    ap.add_argument("--profile-precision", default="fp64", choices=("fp64", "mixed"),
                    help="precision of the --profile-only run")
    ap.add_argument("--profile-mlp", action="store_true",
                    help="run only the warm-start network's training and inference "
                         "timing (for profiler runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    args = ap.parse_args(argv)
    if args.steps < 1 or args.warmup < 0:
        ap.error("--steps must be >= 1 and --warmup >= 0")
    return args


def main(argv=None):
    args = parse_args(argv)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path "
              "(independent flow conditions would go to different GPUs; one cloud "
              "would split into point partitions with halo exchanges)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2406_07441_amd import cloudgen
    from paper_2406_07441_amd import lskum as lk

    torch.cuda.set_device(0)
    if args.profile_mlp:
        print(json.dumps(mlp_profile_run(lk)))
        return
    if args.calibrate_copy:
        src = torch.ones(32 * 2 ** 20, dtype=torch.float64, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    t_setup = time.perf_counter()
    cloud = cloudgen.cloud_2621440()
    gc = lk.Cloud(cloud)
    colours = gc.colours()
    print(f"# cloud n={cloud.n} nnz={cloud.nnz} colours={gc.n_colours} "
          f"degenerate={gc.n_degenerate} setup {time.perf_counter() - t_setup:.1f} s",
          file=sys.stderr, flush=True)
    precisions = [("fp64", lk.FP64)]
    if args.profile_only:
        precisions = [(args.profile_precision, lk.FP64 if args.profile_precision == "fp64"
                       else lk.MIXED)]
    elif not args.no_mixed:
        precisions.append(("mixed", lk.MIXED))
    runs = {}
    for name, prec in precisions:
        elapsed, rep, phases = timed_run(lk, gc, HEAD_MACH, HEAD_AOA, args.steps, args.warmup,
                                         prec, f"timed {name}")
        kern = kernel_rooflines(cloud, colours, phases)
        traffic = measured_traffic(name)
        for k, v in kern.items():
            v["traffic"] = (traffic or {}).get(k)
        ms = 1e3 * elapsed / args.steps
        it_gbs = iteration_bytes(cloud.n) / (ms * 1e-3) / 1e9
        runs[name] = {"seconds": elapsed, "ms_per_step": ms,
                      "point_iters_per_s": cloud.n * args.steps / elapsed,
                      "res_final": rep.res_final, "res_fs": rep.res_fs, "phases_ms": phases,
                      "kernels": kern,
                      "iteration_bandwidth": {"bytes_per_iteration": iteration_bytes(cloud.n),
                                              "achieved_gbs": it_gbs, "peak_gbs": PEAK_HBM_GBS,
                                              "frac": it_gbs / PEAK_HBM_GBS}}
    head = runs[precisions[0][0]]
    dom = max(head["kernels"], key=lambda k: head["kernels"][k]["ms_per_step"])
    roofline = {"kernel": dom, **{k: v for k, v in head["kernels"][dom].items()
                                  if k in ("bound", "achieved", "peak", "unit", "frac",
                                           "traffic")}}
    if args.profile_only:
        print(json.dumps({"ms_per_step": head["ms_per_step"], "phases_ms": head["phases_ms"],
                          "roofline": roofline}))
        return

    extra = {}
    if "mixed" in runs:
        extra["mixed_precision_same_workload"] = {
            **runs["mixed"], "speedup_vs_fp64": runs["fp64"]["seconds"] / runs["mixed"]["seconds"]}

    def leg(name, fn, *a):
        t = time.perf_counter()
        extra[name] = fn(*a)
        print(f"# {name} ({time.perf_counter() - t:.1f} s): {json.dumps(extra[name])}",
              file=sys.stderr, flush=True)

    if args.tol_iters > 0:
        c2 = cloudgen.cloud_163840()
        g2 = lk.Cloud(c2)

        def tol_legs():
            return {"workload": "640x256=163840 pts O-grid, 4% jittered, M0.85 AoA1, limiter K5",
                    "exact_fp64": time_to_tol(lk, g2, args.tol_iters),
                    "fluxdiff_fp64": time_to_tol(lk, g2, args.tol_iters,
                                                 jvp_mode=lk.JVP_FLUXDIFF),
                    "exact_mixed": time_to_tol(lk, g2, args.tol_iters, precision=lk.MIXED)}
        leg("time_to_1e-8_163840", tol_legs)
        leg("explicit_vs_implicit_163840_2000_iters", explicit_vs_implicit, lk, g2, 2000)
        g2.close()
    if args.batch_iters > 0:
        leg("batch_64_conditions", batch_run, lk, cloudgen, args.batch_iters)
    if args.batch_converge_iters > 0:
        leg("batch_64_to_1e-8", batch_converge, lk, cloudgen, args.batch_converge_iters,
            args.batch_converge_seconds)
    if args.histories:
        leg("residual_histories_6400", residual_histories, lk, cloudgen)
    if args.config3_iters > 0:
        leg("cloud_2621440_to_1e-8", config3_run, lk, cloudgen, args.config3_iters,
            args.config3_precisions.split(","))
    if args.warm_steps > 0:
        leg("warm_start", warm_start_run, lk, cloudgen, args.warm_steps, args.warm_held_out,
            args.warm_scale)
    cpu = None
    if args.cpu_seconds > 0:
        t = time.perf_counter()
        cpu = cpu_baseline(cloud, HEAD_MACH, HEAD_AOA, args.cpu_seconds)
        print(f"# cpu baseline ({time.perf_counter() - t:.1f} s): {json.dumps(cpu)}",
              file=sys.stderr, flush=True)

    line = {
        "metric": "point-iters/s + time to 1e-8 res drop: exact-JVP LU-SGS FP64 vs mixed+batched",
        "value": head["point_iters_per_s"], "unit": "point-iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "O-grid cloud 2560x1024=2621440 pts around a 12% symmetric "
                               "profile, M0.5 AoA3, exact-JVP LU-SGS FP64, CFL100, 1 inner "
                               "iteration, limiter K5",
                   "points": cloud.n, "edges": cloud.nnz, "colours": gc.n_colours},
        "roofline": roofline, "roofline_kernels": head["kernels"], "cpu_baseline": cpu,
        "iteration_bandwidth": head["iteration_bandwidth"], "phases_ms": head["phases_ms"],
        **extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
