"""Pins of the oracle's explicit solver (forward Euler in time, U - dt R, with
the implicit scheme's local time step).

* Uniform flow is a fixed point, bitwise (R == 0, also with a flat wall).
* The explicit and implicit schemes share their fixed point: from a state the
  implicit solver has converged (to 1e-10 of the free-stream residual), one
  explicit step changes U by less than 1e-8 of the change of the first explicit
  step from the free stream.
* At CFL 0.4 the explicit iteration is stable and reduces the residual, more
  slowly per iteration than the implicit one.
"""
import numpy as np

import oracle as O
from paper_2406_07441_amd import cloudgen as cg


def test_uniform_flow_is_fixed_point():
    for wall in (False, True):
        c = cg.box(9, 8, h=0.13, wall_bottom=wall)
        o = O.Oracle(c, mach=0.5, aoa_deg=0.0 if wall else 20.0, cfl=0.4)
        U = o.free_stream()
        U1, R, res = o.explicit_iteration(U)
        assert res == 0.0 and np.array_equal(U1, U)


def test_shares_the_implicit_fixed_point():
    c = cg.ogrid(48, 12, r=None)
    oi = O.Oracle(c, mach=0.5, aoa_deg=2.0, cfl=100.0)
    U, it, hist = oi.solve(oi.free_stream(), 3000, tol_abs=1e-12 * 1.0)
    _, res_fs = oi.residual(oi.free_stream())
    assert hist[-1] < 1e-10 * res_fs
    oe = O.Oracle(c, mach=0.5, aoa_deg=2.0, cfl=0.4)
    U1, R, res = oe.explicit_iteration(U)
    Ufs = oe.free_stream()
    step_fs = np.abs(oe.explicit_iteration(Ufs)[0] - Ufs).max()
    assert np.abs(U1 - U).max() < 1e-8 * step_fs


def test_explicit_is_stable_and_slower_than_implicit():
    c = cg.ogrid(48, 12, r=None)
    oe = O.Oracle(c, mach=0.5, aoa_deg=2.0, cfl=0.4)
    oi = O.Oracle(c, mach=0.5, aoa_deg=2.0, cfl=100.0)
    U0 = oe.free_stream()
    _, r0 = oe.residual(U0)
    Ue, Ui = U0, U0
    for _ in range(200):
        Ue, _, re = oe.explicit_iteration(Ue)
        Ui, _, _, ri = oi.iteration(Ui)
    assert np.isfinite(re) and re < 0.5 * r0
    assert ri < re
