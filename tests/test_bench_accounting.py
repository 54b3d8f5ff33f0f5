"""The benchmark's algorithmic work counts (the basis of its roofline figures),
checked against brute-force counts on a small O-grid cloud, and its command
line as the benchmark driver calls it (CPU only)."""
import os
import sys

import numpy as np
import pytest

import oracle as O
from paper_2406_07441_amd import cloudgen as cg

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def small_case():
    cloud = cg.ogrid(48, 12)
    colours = O.Oracle(cloud, mach=0.5, aoa_deg=0.0).colours
    return cloud, colours


def test_sweep_points_exclude_the_fused_and_identity_phases():
    cloud, col = small_case()
    fwd, bwd, launches = bench.sweep_points(col)
    top = col.max()
    assert fwd == sum(1 for p in range(cloud.n) if col[p] > 0)
    assert bwd == sum(1 for p in range(cloud.n) if col[p] < top)
    assert launches == top  # colour 0 inside the residual kernel, the top colour skipped


def test_phase_bytes_follow_the_per_point_table():
    # q, q_x, q_y and the CSR of a 24-neighbour stencil, each read or written once
    assert bench.QGRAD_FIRST_B == 32 + 16 + 100 + 96
    assert bench.QGRAD_INNER_B == 96 + 16 + 100 + 64
    assert bench.RESIDUAL_B == 96 + 16 + 100 + 32 + 32 + 16 + 96 + 2
    assert bench.SWEEP_FWD_B == 32 + 8 + 100 + 16 + 96 + 32 + 32 + 4
    assert bench.SWEEP_BWD_B == 32 + 8 + 100 + 16 + 96 + 32
    n = 1000
    assert bench.iteration_bytes(n) == n * (244 + 276 + 64 + 390 + 8 + 320 + 284 + 128)
    assert bench.iteration_bytes(n, inner=3, limiter=False) == n * (244 + 3 * 276 + 390 + 8
                                                                    + 320 + 284 + 128)


def test_kernel_rooflines_divide_work_by_launch_time():
    cloud, col = small_case()
    phases = {"q_derivatives": 0.02, "residual": 0.05, "norm": 0.004, "forward_sweep": 0.03,
              "backward_sweep": 0.03, "update": 0.002}
    k = bench.kernel_rooflines(cloud, col, phases)
    fwd, _, launches = bench.sweep_points(col)
    f = k["k_sweep forward"]
    assert f["launches_per_step"] == launches
    assert np.isclose(f["achieved"], fwd * bench.SWEEP_FWD_B / 0.03e-3 / 1e9)
    assert np.isclose(f["frac"], f["achieved"] / 8000.0)
    r = k["k_residual"]
    assert r["bound"] == "alu" and np.isclose(r["achieved"],
                                              bench.residual_flops(cloud) / 0.05e-3 / 1e12)


def test_residual_flops_per_point():
    cloud, _ = small_case()
    deg = np.diff(cloud.nbr_off)
    want = 0.0
    for p in range(cloud.n):
        if cloud.type[p] == cg.OUTER:
            continue
        splits = 2.0 if cloud.type[p] == cg.INTERIOR else 1.5
        want += deg[p] * (bench.NB_OPS + splits * bench.SPLIT_OPS)
    assert bench.residual_flops(cloud) == want
    # an interior point with the full 5 x 5 ring: 24 x (140 + 2 x 161)
    assert bench.NB_OPS == 140 and bench.SPLIT_OPS == 161
    assert 24 * (bench.NB_OPS + 2 * bench.SPLIT_OPS) == 11088


def test_driver_command_line_is_accepted():
    # the driver's own invocation; any positive step count and any warm-up
    a = bench.parse_args(["--gpus", "1", "--steps", "20", "--warmup", "5"])
    assert (a.gpus, a.steps, a.warmup) == (1, 20, 5)
    for steps, warmup in ((7, 0), (1, 3), (400, 40)):
        a = bench.parse_args(["--steps", str(steps), "--warmup", str(warmup)])
        assert bench.check_every_for(steps) >= 1 and steps % bench.check_every_for(steps) == 0
    assert bench.check_every_for(20) == 20 and bench.check_every_for(200) == 40
    with pytest.raises(SystemExit):
        bench.parse_args(["--steps", "0"])


def test_more_than_one_gpu_exits_with_a_message(capsys):
    with pytest.raises(SystemExit) as ei:
        bench.main(["--gpus", "2"])
    assert ei.value.code == 2
    assert "one GPU" in capsys.readouterr().err
