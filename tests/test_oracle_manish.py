"""Pins of the oracle's Manish et al. variant (eq. 29-33, 36-38).

* The unsplit Jacobian product equals the sum of the two split products
  (A = A+ + A-, since G = G+ + G-), exact and as flux differences.
* On a symmetric stencil (interior points of a uniform box) S vanishes for any
  increment, and the scalar diagonal has the closed form
  D = 1/dt + 0.6 (|u1| + a + |u2| + a) / h (the 5 x 5 ring: LS_x+-(1) = -+0.6/h).
* At rest the spectral part of the Manish diagonal (rho(A)/2 = a/2 per split)
  is exactly half of the Anandhanarayanan one (rho(A+-) = a).
* With a zero previous increment the Manish iteration is the colour sweep
  with its own diagonal and S = 0; with the previous increment S enters the
  forward right-hand side as R - S.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2406_07441_amd import cloudgen as cg


def rand_state(rng):
    rho = rng.uniform(0.5, 1.5)
    u = rng.uniform(-0.9, 0.9, 2)
    p = rng.uniform(0.4, 1.2)
    E = p / 0.4 + 0.5 * rho * (u @ u)
    return np.array([rho, rho * u[0], rho * u[1], E])


@pytest.mark.parametrize("mode", [0, 1])
def test_unsplit_product_is_sum_of_split_products(mode):
    rng = np.random.default_rng(5)
    for _ in range(20):
        U = rand_state(rng)
        dU = rng.standard_normal(4) * (1e-7 if mode else 1.0)
        th = rng.uniform(0, 2 * math.pi)
        d = (math.cos(th), math.sin(th))
        J = O.unsplit_jvp(U, dU, d, jvp_mode=mode)
        Js = O.flux_jvp(U, dU, d, +1, jvp_mode=mode) + O.flux_jvp(U, dU, d, -1, jvp_mode=mode)
        # flux differences of O(1) fluxes lose ~1e-16 absolute to cancellation
        tol = dict(rtol=1e-9, atol=1e-12 * np.abs(J).max()) if mode == 0 else \
            dict(rtol=1e-6, atol=1e-14)
        assert np.allclose(J, Js, **tol)


def box_case(variant):
    c = cg.box(11, 11, h=0.1)
    o = O.Oracle(c, mach=0.5, aoa_deg=30.0, cfl=10.0, inner_iters=1, variant=variant)
    return c, o


def test_symmetric_stencil_source_vanishes_and_diagonal_closed_form():
    c, o = box_case(O.MANISH)
    rng = np.random.default_rng(2)
    U = o.free_stream()
    dU = rng.standard_normal((4, c.n))
    S = o.manish_source(U, dU)
    # interior points whose 5 x 5 ring lies inside the box
    jj, kk = np.arange(c.n) % 11, np.arange(c.n) // 11
    inner = (jj >= 2) & (jj <= 8) & (kk >= 2) & (kk <= 8)
    assert np.abs(S[:, inner]).max() < 1e-12 * np.abs(dU).max()
    assert np.abs(S[:, ~inner & (c.type == 1)]).max() > 1e-6   # one-sided stencils
    dt, D = o.timestep_diag(U)
    a = 1.0
    u1, u2 = 0.5 * math.cos(math.radians(30)), 0.5 * math.sin(math.radians(30))
    want = 1.0 / dt + 0.6 * ((abs(u1) + a) + (abs(u2) + a)) / 0.1
    assert np.allclose(D[inner], want[inner], rtol=1e-12)


@pytest.mark.parametrize("aoa", [0.0, 180.0, 30.0])
def test_anandh_diagonal_with_supersonic_split_velocity(aoa):
    # eq. (34)-(35): rho(A+) = max(u_d + a, 0), rho(A-) = max(a - u_d, 0); on the
    # symmetric 5 x 5 ring of a uniform box LS_d+(1) = -0.6/h, LS_d-(1) = +0.6/h,
    # so D = 1/dt + 0.6/h sum_d [max(u_d + a, 0) + max(a - u_d, 0)].  At M 1.5 the
    # split velocity exceeds the speed of sound and one half vanishes
    # (|u_d + a| or |a - u_d| would not).
    c = cg.box(11, 11, h=0.1)
    o = O.Oracle(c, mach=1.5, aoa_deg=aoa, cfl=10.0, variant=O.ANANDH)
    U = o.free_stream()
    dt, D = o.timestep_diag(U)
    a = 1.0
    u1, u2 = 1.5 * math.cos(math.radians(aoa)), 1.5 * math.sin(math.radians(aoa))
    spec = sum(max(u + a, 0.0) + max(a - u, 0.0) for u in (u1, u2))
    jj, kk = np.arange(c.n) % 11, np.arange(c.n) // 11
    inner = (jj >= 2) & (jj <= 8) & (kk >= 2) & (kk <= 8)
    assert np.allclose(D[inner], 1.0 / dt[inner] + 0.6 / 0.1 * spec, rtol=1e-12)
    if aoa == 0.0:   # u1 = 1.5 > a: the x- half contributes nothing
        assert spec == pytest.approx((1.5 + a) + 0.0 + 2 * a)
    # dt = CFL h / (|u| + a)
    assert np.allclose(dt[inner], 10.0 * 0.1 / (1.5 + a), rtol=1e-14)


def test_diagonals_at_rest():
    # at rest rho(A+) = rho(A-) = a (Anandhanarayanan) and rho(A)/2 = a/2 (Manish):
    # the spectral parts of the two diagonals differ by exactly a factor 2
    c = cg.box(11, 11, h=0.1)
    oa = O.Oracle(c, mach=1e-300, aoa_deg=0.0, cfl=10.0, variant=O.ANANDH)
    om = O.Oracle(c, mach=1e-300, aoa_deg=0.0, cfl=10.0, variant=O.MANISH)
    U = oa.free_stream()
    dt, Da = oa.timestep_diag(U)
    _, Dm = om.timestep_diag(U)
    act = c.type != 2
    assert np.allclose(Dm[act] - 1 / dt[act], 0.5 * (Da[act] - 1 / dt[act]), rtol=1e-12)
    assert np.all(Dm[act] > 1 / dt[act])


def test_forward_rhs_is_R_minus_S():
    c = cg.ogrid(48, 12)
    o = O.Oracle(c, mach=0.6, aoa_deg=2.0, variant=O.MANISH)
    U0 = o.free_stream()
    U1, R1, dU1, _ = o.iteration(U0)                 # S = 0 (no previous increment)
    dt, D = o.timestep_diag(U0)
    assert np.allclose(dU1, o.lusgs(U0, R1, D), rtol=0, atol=1e-15)
    U2, R2, dU2, _ = o.iteration(U1, dU1)
    S = o.manish_source(U1, dU1)
    assert np.abs(S).max() > 0
    _, D1 = o.timestep_diag(U1)
    assert np.allclose(dU2, o.lusgs(U1, R2 - S, D1), rtol=0, atol=1e-15)


def test_manish_converges_on_subsonic_cloud():
    # with S lagged one iteration the explicit part limits the time step: the
    # 96 x 32 cloud converges at CFL 5 (and goes non-physical at CFL 20-100),
    # faster than the Anandhanarayanan variant at the same CFL
    c = cg.ogrid(96, 32, r=None)
    drops = {}
    for variant in (O.MANISH, O.ANANDH):
        o = O.Oracle(c, mach=0.5, aoa_deg=2.0, cfl=5.0, variant=variant)
        U = o.free_stream()
        _, res0 = o.residual(U)
        U, it, hist = o.solve(U, 300)
        assert it == 300 and np.all(np.isfinite(hist))
        drops[variant] = hist[-1] / res0
    assert drops[O.MANISH] < 1e-2 and drops[O.MANISH] < drops[O.ANANDH]
