#!/usr/bin/env python3
"""Benchmark of the implicit LSKUM hot path on one MI355X.

Workload (the timed steps): the transonic NACA 0012-type case -- a
640 x 256 = 163,840-point O-grid cloud with 4% of interior points jittered
(seed 2406), Mach 0.85, AoA 1 deg; exact-JVP modified LU-SGS in FP64, CFL 100,
one inner iteration of the q-derivatives, Venkatakrishnan limiter (K = 5) on
the q~ reconstruction (the shock needs it to converge; the paper names none).
A step is one implicit iteration: q-derivatives, limiter, residual, forward
and backward colour sweeps, state update.  ``value`` is point-iterations per
second over the timed steps (HIP-graph replay, inputs resident in HBM).

Also reported: per-phase GPU times from HIP events, the roofline of the
dominant kernel, time to a 1e-8 residual drop with exact and flux-difference
Jacobian products (FP64) and with mixed precision, the batched 64-condition
workload, and the CPU oracle's rate on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MACH, AOA, CFL, INNER, LIMITER, LIMITER_K = 0.85, 1.0, 100.0, 1, 1, 5.0

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6

# Algorithmic FP64 operation count of the residual, with elementary functions
# costed at the operation count of a standard software evaluation.
COST = {"exp": 14, "erf": 26, "sqrt": 8, "div": 8, "log": 20}
# per neighbour: dx, dy; two q~ reconstructions (4 x 5 each); two q~ -> primitive
# conversions (11 arithmetic + exp + sqrt + 2 div each)
NB_OPS = 2 + 40 + 2 * (11 + COST["exp"] + COST["sqrt"] + 2 * COST["div"])
# per (neighbour, split): weight (3), two split fluxes (25 arithmetic + erf + exp
# + div each), difference, scale and accumulate (12)
SPLIT_OPS = 3 + 2 * (25 + COST["erf"] + COST["exp"] + COST["div"]) + 12

# Algorithmic bytes of the sweep, each array read or written once. Per swept
# point: colour-sorted index 4, list offset 4, component 4, type 1, wall
# frame 16, D 8, own R (forward) or dU* (backward) 32, result 32, and its
# linearisation records ((rho, u1, u2, p) 32 and the erf/exp pairs 32) and
# increment (32) as read by its neighbours; per list entry: neighbour index
# 4, split weights 16, split code 1.
SWEEP_POINT_BYTES = 4 + 4 + 4 + 1 + 16 + 8 + 32 + 32 + 64 + 32
SWEEP_ENTRY_BYTES = 4 + 16 + 1
# the same in mixed precision (fp32 D, increments, records and weights; R stays fp64)
SWEEP_POINT_BYTES_F32 = 4 + 4 + 4 + 1 + 16 + 4 + 32 + 16 + 32 + 16
SWEEP_ENTRY_BYTES_F32 = 4 + 8 + 1


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


def forward_sweep_bytes(cloud, colours, mixed: bool = False) -> tuple[float, int]:
    """Algorithmic bytes of the forward sweep's colour-phase launches and their
    number: colours 1 and up (the colour-0 phase has no lower neighbours and is
    formed inside the residual kernel), with every lower-list entry."""
    import numpy as np
    deg = np.diff(cloud.nbr_off)
    src = np.repeat(np.arange(cloud.n), deg)
    lower = int(np.count_nonzero(colours[cloud.nbr_idx] < colours[src]))
    swept = int(np.count_nonzero(colours > 0))
    pb, eb = ((SWEEP_POINT_BYTES_F32, SWEEP_ENTRY_BYTES_F32) if mixed
              else (SWEEP_POINT_BYTES, SWEEP_ENTRY_BYTES))
    return float(swept * pb + lower * eb), int(colours.max())


def iteration_bytes(cloud, colours, mixed: bool = False) -> float:
    """Algorithmic bytes of one whole iteration (m = 1 with the limiter), each
    array read or written once, neighbour data counted once per pass:
    q-derivative pass 0 (q 32, xy 16, offsets 8, LS matrix 32, 4 per stencil
    entry, q_x/q_y write 64), the limited inner pass (q, q_x, q_y 96, xy 16,
    offsets 8, LS matrix 32, 4 per entry, four derivative writes 128), the
    residual (q, limited q_x, q_y 96, xy 16, frame 16, type 1, offsets 8,
    split and diagonal coefficients 128, U 32, 4 per entry; R 32, R_rho^2 8,
    linearisation records 64 and D 8 written, or 32 and 4 in mixed precision),
    the norm (8), both sweeps as above and the update (U read and written 64,
    dU 32 or 16, q written 32)."""
    import numpy as np
    deg = np.diff(cloud.nbr_off).astype(np.int64)
    src = np.repeat(np.arange(cloud.n), deg)
    lower = int(np.count_nonzero(colours[cloud.nbr_idx] < colours[src]))
    upper = cloud.nnz - lower
    if mixed:
        per_point = 152 + 280 + 373 + 8 + 2 * SWEEP_POINT_BYTES_F32 + 112
        entry = SWEEP_ENTRY_BYTES_F32
    else:
        per_point = 152 + 280 + 409 + 8 + 2 * SWEEP_POINT_BYTES + 128
        entry = SWEEP_ENTRY_BYTES
    return float(cloud.n * per_point + 3 * 4 * cloud.nnz + entry * (lower + upper))


def large_cloud_run(lk, cloudgen, steps: int):
    """The 2,621,440-point cloud (M 0.5, AoA 3 deg, the benchmark's solver
    settings), FP64 and mixed precision: graph-replayed iterations from the
    free stream, HIP-event phase times and the bandwidth figures; its working
    set is larger than the 256 MB Infinity Cache."""
    cloud = cloudgen.cloud_2621440()
    gc = lk.Cloud(cloud)
    colours = gc.colours()
    flops = residual_flops(cloud)
    out = {"points": cloud.n, "edges": cloud.nnz, "colours": gc.n_colours}
    for name, prec in (("fp64", lk.FP64), ("mixed", lk.MIXED)):
        it_bytes = iteration_bytes(cloud, colours, mixed=prec == lk.MIXED)
        fwd_b, fwd_launches = forward_sweep_bytes(cloud, colours, mixed=prec == lk.MIXED)
        prm = lk.default_params(cfl=CFL, inner_iters=INNER, precision=prec, check_every=10,
                                tol_rel=0.0, max_iters=10, limiter=LIMITER, limiter_k=LIMITER_K)
        st = lk.State(gc, 0.5, 3.0, prm)
        st.solve()
        prm.max_iters = steps
        st.set_params(prm)
        rep = st.solve()
        ms = 1e3 * rep.seconds / rep.iters
        acc = None
        for _ in range(10):
            ph = st.step_timed()
            acc = ph if acc is None else {k: acc[k] + ph[k] for k in acc}
        phases = {k: v / 10 for k, v in acc.items()}
        st.close()
        sweep_gbs = fwd_b / (phases["forward_sweep"] * 1e-3) / 1e9
        it_gbs = it_bytes / (ms * 1e-3) / 1e9
        out[name] = {
            "iters": rep.iters, "ms_per_iter": ms, "iteration_bytes": it_bytes,
            "point_iters_per_s": cloud.n / (ms * 1e-3), "phases_ms": phases,
            "iteration_gbs": it_gbs, "iteration_frac_hbm": it_gbs / PEAK_HBM_GBS,
            "forward_sweep_gbs": sweep_gbs, "forward_sweep_frac_hbm": sweep_gbs / PEAK_HBM_GBS,
            "forward_sweep_launches": fwd_launches,
            "residual_tflops": flops / (phases["residual"] * 1e-3) / 1e12}
        print(f"# 2.6M {name}: {ms:.3f} ms/iteration, whole iteration {it_gbs:.0f} GB/s, "
              f"forward sweep {sweep_gbs:.0f} GB/s", file=sys.stderr, flush=True)
    return out


def device_source_hash() -> str:
    src = os.path.join(ROOT, "paper_2406_07441_amd", "csrc", "lskum_device.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from rocprofv3 FETCH_SIZE/WRITE_SIZE counter runs,
    when the summary in profiles/ was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_163840_transonic_fp64.md")
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
    # algorithmic bytes: each condition's iterations on its own cloud (mixed precision)
    cb = [iteration_bytes(c, g.colours(), mixed=True) for c, g in zip(clouds, gcs)]
    moved = sum(r["iters"] * cb[k % 8] for k, r in enumerate(reps))
    out = {"conditions": 64, "clouds": [c.n for c in clouds], "points": b.n_points,
           "colour_phases": b.n_colours, "iters": iters, "seconds": tot,
           "point_iters_per_s": pts / tot, "iteration_gbs": moved / tot / 1e9,
           "iteration_frac_hbm": moved / tot / 1e9 / PEAK_HBM_GBS,
           "lanes": {"sweep": lanes[0], "residual": lanes[1]},
           "failed": int(sum(r["status"] == lk.ERR_NONPHYSICAL for r in reps)),
           "median_res_drop": float(np.median([r["res_final"] / r["res_fs"] for r in reps]))}
    b.close()
    return out


CHUNK_ITERS = 2000   # long solves run in chunks, each printing a progress line


def solve_chunked(obj, prm, max_iters, n_cond, label):
    """Solves a State (n_cond 1) or Batch to its tolerance in chunks of
    CHUNK_ITERS iterations; returns per-condition (iters, seconds, status, cl,
    cd) at first convergence and the total seconds."""
    done = [None] * n_cond
    total_it, total_s = 0, 0.0
    last = None
    while total_it < max_iters and any(d is None for d in done):
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
                           "status": 0, "cl": r["cl"], "cd": r["cd"],
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
                       "cl": last[k]["cl"], "cd": last[k]["cd"],
                       "res_drop": last[k]["res_final"] / last[k]["res_fs"]}
    return done, total_s


def batch_converge(lk, cloudgen, max_iters):
    """The 64-condition batch solved to 1e-8 of each condition's free-stream
    residual: time until all retire, per-condition iterations."""
    import numpy as np
    clouds = cloudgen.batch_clouds()
    gcs = [lk.Cloud(c) for c in clouds]
    mach, aoa = cloudgen.batch_conditions()
    prm = lk.default_params(cfl=CFL, inner_iters=INNER, precision=lk.MIXED, limiter=LIMITER,
                            limiter_k=LIMITER_K, check_every=100, tol_rel=1e-8)
    b = lk.Batch(gcs, np.arange(64) % 8, mach, aoa, prm)
    lanes = b.autotune(2)
    prm.sweep_lanes, prm.residual_lanes = lanes[0], lanes[1]
    done, tot = solve_chunked(b, prm, max_iters, 64, "batch to 1e-8")
    pts = sum(d["iters"] * b.sizes[k] for k, d in enumerate(done))
    out = {"conditions": 64, "points": b.n_points,
           "seconds_until_all_retired": max(d["seconds"] for d in done),
           "point_iters_per_s": pts / tot, "lanes": {"sweep": lanes[0], "residual": lanes[1]},
           "iters": [d["iters"] for d in done],
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


def warm_start_run(lk, cloudgen, train_steps: int, held_out: int):
    """Learned warm start, scaled down from the 640k-point / 512-field recipe:
    converged fields of 32 conditions on 4 clouds of 20k-60k points (mixed
    precision, to 1e-6) train the network; `held_out` conditions on a held-out
    640 x 256 cloud are then solved to 1e-8 of each condition's free-stream
    residual three ways: the plain FP64 solver one condition at a time from the
    free stream (baseline); the mixed-precision batch from the free stream; the
    mixed-precision batch from the warm start."""
    import numpy as np
    import torch
    clouds = cloudgen.batch_clouds(seed=40, count=4, nmin=20_000, nmax=60_000)
    gcs = [lk.Cloud(c) for c in clouds]
    mach, aoa = cloudgen.batch_conditions(seed=41, count=32)
    prm = lk.default_params(cfl=CFL, inner_iters=INNER, precision=lk.MIXED, limiter=LIMITER,
                            limiter_k=LIMITER_K, check_every=50, tol_rel=1e-6, max_iters=40000)
    t0 = time.perf_counter()
    b = lk.Batch(gcs, np.arange(32) % 4, mach, aoa, prm)
    reps, _ = b.solve()
    ok = [r["status"] == 0 for r in reps]
    X, T = b.features(targets=True)
    # rows of conditions that did not converge are left out of the training set
    keep = torch.cat([torch.full((b.sizes[k],), bool(ok[k]), device="cuda") for k in range(32)])
    X, T = X[keep].contiguous(), T[keep].contiguous()
    b.close()
    gen_s = time.perf_counter() - t0
    print(f"# warm start: {int(sum(ok))}/32 training fields in {gen_s:.1f} s", file=sys.stderr,
          flush=True)
    net = lk.MLP(seed=11, max_rows=8192)
    hist, train_s = net.train(X, T, steps=train_steps, batch=8192, lr=3e-3, lr_final=1e-5, seed=13)
    rows = X.shape[0]
    print(f"# warm start: trained {train_steps} steps in {train_s:.1f} s", file=sys.stderr,
          flush=True)

    held = cloudgen.ogrid(640, 256, r=None, t=0.12, name="heldout640x256")
    gh = lk.Cloud(held)
    hm, ha = cloudgen.batch_conditions(seed=42, count=held_out)
    common = dict(cfl=CFL, inner_iters=INNER, limiter=LIMITER, limiter_k=LIMITER_K,
                  check_every=50, tol_rel=1e-8, max_iters=60000)
    # (a) baseline: plain FP64 solver, one condition at a time, free-stream start
    base = []
    for m, a_ in zip(hm, ha):
        st = lk.State(gh, float(m), float(a_), lk.default_params(**common))
        r = st.solve()
        base.append(r.as_dict())
        st.close()
    base_s = sum(r["seconds"] for r in base)
    print(f"# warm start: FP64 baseline {base_s:.1f} s", file=sys.stderr, flush=True)
    cc = np.zeros(held_out, np.int32)
    prm_mx = lk.default_params(precision=lk.MIXED, **common)
    # (b) mixed-precision batch, free-stream start
    bf = lk.Batch([gh], cc, hm, ha, prm_mx)
    r_bf, t_bf = bf.solve()
    bf.close()
    # (c) mixed-precision batch, warm start (inference and residual check inside the timing)
    bw = lk.Batch([gh], cc, hm, ha, prm_mx)
    Xh = bw.features()
    torch.cuda.synchronize()
    ti = time.perf_counter()
    net.forward(Xh)
    torch.cuda.synchronize()
    infer_s = time.perf_counter() - ti
    tw = time.perf_counter()
    fb, res_w = net.warm_start(bw)
    warm_s = time.perf_counter() - tw
    r_bw, t_bw = bw.solve()
    bw.close()
    net.close()
    return {
        "training": {"clouds": [c.n for c in clouds], "conditions": 32,
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


def cpu_baseline(cloud, iters: int):
    import oracle
    o = oracle.Oracle(cloud, mach=MACH, aoa_deg=AOA, cfl=CFL, inner_iters=INNER,
                      limiter=LIMITER, limiter_k=LIMITER_K)
    U = o.free_stream()
    t0 = time.perf_counter()
    for _ in range(iters):
        U, _, _, _ = o.iteration(U)
    dt = time.perf_counter() - t0
    return {"value": cloud.n * iters / dt, "unit": "point-iters/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} serial FP64 oracle iterations of the {cloud.n}-point workload "
                      f"from the free-stream start ({dt:.1f} s) on one core of {host_cpu()}"}


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--tol-iters", type=int, default=60000,
                    help="iteration cap of the time-to-1e-8 runs (0 skips them)")
    ap.add_argument("--batch-iters", type=int, default=200,
                    help="iterations of the 64-condition batch run (0 skips it)")
    ap.add_argument("--cpu-iters", type=int, default=4, help="oracle iterations (0 skips)")
    ap.add_argument("--warm-steps", type=int, default=6000,
                    help="training steps of the warm-start leg (0 skips it)")
    ap.add_argument("--warm-held-out", type=int, default=4,
                    help="held-out conditions of the warm-start leg")
    ap.add_argument("--batch-converge-iters", type=int, default=0,
                    help="solve the 64-condition batch to 1e-8 with this cap (0 skips)")
    ap.add_argument("--large-steps", type=int, default=200,
                    help="graph-replayed iterations of the 2,621,440-point bandwidth leg (0 skips)")
    ap.add_argument("--config3-iters", type=int, default=0,
                    help="2,621,440-point FP64 vs mixed run to 1e-8 with this cap (0 skips)")
    ap.add_argument("--config3-precisions", default="fp64,mixed",
                    help="precisions of the --config3-iters leg (comma separated)")
    ap.add_argument("--profile-only", action="store_true",
                    help="run only the timed steps (for profiler runs)")
    ap.add_argument("--profile-mlp", action="store_true",
                    help="run only the warm-start network's training and inference "
                         "timing (for profiler runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path "
              "(independent flow conditions would go to different GPUs; one cloud "
              "would split into point partitions with halo exchanges)", file=sys.stderr)
        sys.exit(2)
    if args.steps % 10 or args.warmup % 10:
        print("--steps and --warmup must be multiples of 10", file=sys.stderr)
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
    cloud = cloudgen.cloud_163840()
    gc = lk.Cloud(cloud)
    # host readback of the residual every 40 iterations when the step counts allow
    # (the convergence test itself runs on the device after every iteration)
    every = 40 if args.steps % 40 == 0 and args.warmup % 40 == 0 else 10
    prm = params(lk, check_every=every, tol_rel=0.0, max_iters=args.warmup)
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
    st.close()
    ncol = gc.n_colours
    traffic = measured_traffic()
    flops = residual_flops(cloud)
    res_ms = phases["residual"]
    res_tf = flops / (res_ms * 1e-3) / 1e12
    fwd_b, fwd_launches = forward_sweep_bytes(cloud, gc.colours())
    sweep_ms = phases["forward_sweep"] / fwd_launches  # average launch of a colour phase
    sweep_b = fwd_b / fwd_launches                     # algorithmic bytes per launch
    sweep_gbs = sweep_b / (sweep_ms * 1e-3) / 1e9
    kernels = {
        "k_sweep_forward": {"bound": "hbm", "achieved": sweep_gbs, "peak": PEAK_HBM_GBS,
                            "unit": "GB/s", "frac": sweep_gbs / PEAK_HBM_GBS,
                            "traffic": (traffic or {}).get("k_sweep_forward"),
                            "bytes_per_launch": sweep_b, "avg_ms": sweep_ms,
                            "launches_per_step": fwd_launches,
                            "ms_per_step": phases["forward_sweep"]},
        "k_residual": {"bound": "alu", "achieved": res_tf, "peak": PEAK_FP64_TFLOPS,
                       "unit": "TFLOP/s", "frac": res_tf / PEAK_FP64_TFLOPS,
                       "traffic": (traffic or {}).get("k_residual"),
                       "flops_per_launch": flops, "avg_ms": res_ms, "launches_per_step": 1,
                       "ms_per_step": res_ms},
    }
    # the two q-derivative passes together (algorithmic bytes as in iteration_bytes)
    # and the update, both against HBM
    qg_b = float(cloud.n * (152 + 280) + 2 * 4 * cloud.nnz)
    qg_gbs = qg_b / (phases["q_derivatives"] * 1e-3) / 1e9
    up_b = float(cloud.n * 128)
    up_gbs = up_b / (phases["update"] * 1e-3) / 1e9
    others = {
        "k_qgrad (both passes)": {"bound": "hbm", "achieved": qg_gbs, "peak": PEAK_HBM_GBS,
                                  "unit": "GB/s", "frac": qg_gbs / PEAK_HBM_GBS,
                                  "bytes_per_step": qg_b, "launches_per_step": 2,
                                  "ms_per_step": phases["q_derivatives"]},
        "k_update": {"bound": "hbm", "achieved": up_gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": up_gbs / PEAK_HBM_GBS, "traffic": (traffic or {}).get("k_update"),
                     "bytes_per_launch": up_b, "launches_per_step": 1,
                     "ms_per_step": phases["update"]},
    }
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    kernels.update(others)
    it_bytes = iteration_bytes(cloud, gc.colours())
    it_gbs = it_bytes / (ms_per_step * 1e-3) / 1e9
    iteration_bw = {"bytes_per_iteration": it_bytes, "achieved_gbs": it_gbs,
                    "peak_gbs": PEAK_HBM_GBS, "frac": it_gbs / PEAK_HBM_GBS}
    roofline = {"kernel": dom, **{k: v for k, v in kernels[dom].items()
                                  if k in ("bound", "achieved", "peak", "unit", "frac", "traffic")}}
    if args.profile_only:
        print(json.dumps({"ms_per_step": ms_per_step, "phases_ms": phases, "roofline": roofline}))
        return

    extra = {}
    if args.tol_iters > 0:
        extra["time_to_1e-8"] = {
            "exact_fp64": time_to_tol(lk, gc, args.tol_iters),
            "fluxdiff_fp64": time_to_tol(lk, gc, args.tol_iters, jvp_mode=lk.JVP_FLUXDIFF),
            "exact_mixed": time_to_tol(lk, gc, args.tol_iters, precision=lk.MIXED),
        }
        print(f"# time to tol: {json.dumps(extra['time_to_1e-8'])}", file=sys.stderr, flush=True)
    if args.tol_iters > 0:
        extra["explicit_vs_implicit_2000_iters"] = explicit_vs_implicit(lk, gc, 2000)
        print(f"# explicit vs implicit: {json.dumps(extra['explicit_vs_implicit_2000_iters'])}",
              file=sys.stderr, flush=True)
    if args.batch_iters > 0:
        extra["batch_64_conditions"] = batch_run(lk, cloudgen, args.batch_iters)
        print(f"# batch: {json.dumps(extra['batch_64_conditions'])}", file=sys.stderr, flush=True)
    if args.batch_converge_iters > 0:
        extra["batch_64_to_1e-8"] = batch_converge(lk, cloudgen, args.batch_converge_iters)
        print(f"# batch to 1e-8: {json.dumps(extra['batch_64_to_1e-8'])}", file=sys.stderr,
              flush=True)
    if args.large_steps > 0:
        extra["cloud_2621440_bandwidth"] = large_cloud_run(lk, cloudgen, args.large_steps)
    if args.config3_iters > 0:
        extra["cloud_2621440_to_1e-8"] = config3_run(lk, cloudgen, args.config3_iters,
                                                     args.config3_precisions.split(","))
        print(f"# 2.6M: {json.dumps(extra['cloud_2621440_to_1e-8'])}", file=sys.stderr, flush=True)
    if args.warm_steps > 0:
        extra["warm_start"] = warm_start_run(lk, cloudgen, args.warm_steps, args.warm_held_out)
        print(f"# warm start: {json.dumps(extra['warm_start'])}", file=sys.stderr, flush=True)
    cpu = cpu_baseline(cloud, args.cpu_iters) if args.cpu_iters > 0 else None

    line = {
        "metric": "point-iters/s + time to 1e-8 res drop: exact-JVP LU-SGS FP64 vs mixed+batched",
        "value": value, "unit": "point-iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "O-grid NACA0012-type cloud 640x256=163840 pts, 4% jittered, "
                               "M0.85 AoA1, exact-JVP LU-SGS FP64, CFL100, 1 inner iteration, "
                               "limiter K5",
                   "points": cloud.n, "edges": cloud.nnz, "colours": ncol},
        "roofline": roofline, "roofline_kernels": kernels, "cpu_baseline": cpu,
        "iteration_bandwidth": iteration_bw, "phases_ms": phases, **extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
