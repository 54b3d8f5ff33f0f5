"""The oracle's per-point loops run on OpenMP threads; its results must not
depend on the thread count (each point writes only its own outputs, the sums
over points stay serial)."""
import numpy as np

import oracle as O
from paper_2406_07441_amd import cloudgen as cg


def run(threads, cloud, **kw):
    O.set_threads(threads)
    o = O.Oracle(cloud, **kw)
    U, dU = o.free_stream(), None
    out = []
    for _ in range(3):
        U, R, dU, res = o.iteration(U, dU)
        out += [U.copy(), R.copy(), dU.copy(), res]
    out.append(o.forces(U))
    return out


def test_iterations_are_bitwise_independent_of_the_thread_count():
    keep = O.threads()
    try:
        cases = [(cg.ogrid(64, 16, r=1.15), dict(mach=0.63, aoa_deg=2.0, limiter=1)),
                 (cg.ogrid(64, 16, r=1.15), dict(mach=0.63, aoa_deg=2.0, variant=O.MANISH,
                                                 cfl=5.0, jvp_mode=1)),
                 (cg.ogrid(64, 16, r=1.15), dict(mach=0.5, aoa_deg=1.0, order=O.WALL_FIRST,
                                                 inner_iters=2))]
        for cloud, kw in cases:
            a, b = run(1, cloud, **kw), run(4, cloud, **kw)
            for x, y in zip(a, b):
                assert np.array_equal(np.asarray(x), np.asarray(y))
    finally:
        O.set_threads(keep)
