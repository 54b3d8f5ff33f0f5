"""The benchmark's algorithmic work counts (the basis of its roofline figures),
checked against brute-force counts on a small O-grid cloud (CPU only)."""
import os
import sys

import numpy as np

import oracle as O
from paper_2406_07441_amd import cloudgen as cg

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def small_case():
    cloud = cg.ogrid(48, 12)
    colours = O.Oracle(cloud, mach=0.5, aoa_deg=0.0).colours
    return cloud, colours


def test_forward_sweep_bytes_counts_points_and_lower_entries():
    cloud, col = small_case()
    swept, lower = 0, 0
    for p in range(cloud.n):
        if col[p] > 0:
            swept += 1
        for e in range(cloud.nbr_off[p], cloud.nbr_off[p + 1]):
            lower += col[cloud.nbr_idx[e]] < col[p]
    for mixed, pb, eb in ((False, bench.SWEEP_POINT_BYTES, bench.SWEEP_ENTRY_BYTES),
                          (True, bench.SWEEP_POINT_BYTES_F32, bench.SWEEP_ENTRY_BYTES_F32)):
        b, launches = bench.forward_sweep_bytes(cloud, col, mixed=mixed)
        assert b == swept * pb + lower * eb
        assert launches == col.max()  # colour 0 is formed inside the residual kernel
    assert bench.SWEEP_POINT_BYTES == 197 and bench.SWEEP_ENTRY_BYTES == 21


def test_iteration_bytes_split_the_stencil_once():
    cloud, col = small_case()
    b64 = bench.iteration_bytes(cloud, col)
    b32 = bench.iteration_bytes(cloud, col, mixed=True)
    # every stencil entry appears in exactly one of the lower and upper lists
    per_point = 152 + 280 + 409 + 8 + 2 * bench.SWEEP_POINT_BYTES + 128
    assert b64 == cloud.n * per_point + 12 * cloud.nnz + bench.SWEEP_ENTRY_BYTES * cloud.nnz
    assert b32 < b64


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
