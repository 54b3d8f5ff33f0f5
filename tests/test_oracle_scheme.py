"""Pins of the oracle's meshfree scheme: least squares, q-derivatives,
residual, LU-SGS sweeps, colouring and forces.

Each test checks the oracle against something the paper or the mathematics
fixes, not against a retyped copy of the oracle:
  * LS weights of a split stencil (eq. 11, 13) reproduce d(da)/da = 1 and
    d(db)/da = 0 and are exact on linear fields;
  * the q-derivative inner iteration (eq. 16) keeps the exact derivatives of
    a quadratic field, and pass 0 is exact on linear fields;
  * a uniform flow has R == 0 bitwise (all split-flux differences vanish);
  * R converges to div G at second order (eq. 9-11 defect correction);
  * a mirror-symmetric cloud and state give a mirrored residual;
  * the colour sweeps (eq. 27, Algorithm 6) equal a dense solve of
    (D + U)^-1 D (D + L)^-1 (-R) assembled column by column from the
    Jacobian products;
  * Algorithm 4 colours a hand-traced example exactly and always yields a
    proper colouring;
  * a uniform pressure exerts no force; zero incidence on the symmetric
    profile gives zero lift, subsonic and supersonic (M 1.2, with a shock).
"""
import numpy as np
import pytest

import oracle as O
from paper_2406_07441_amd import cloudgen as cg

GAMMA = 1.4


def prim_field(x, y):
    rho = 1 + 0.1 * np.sin(x) * np.cos(y)
    u = 0.5 + 0.1 * np.cos(x + y)
    v = 0.2 + 0.05 * np.sin(2 * x - y)
    p = 1 / GAMMA + 0.1 * np.cos(x) * np.sin(y)
    return rho, u, v, p


def U_field(x, y):
    rho, u, v, p = prim_field(x, y)
    return np.array([rho, rho * u, rho * v, p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v)])


def euler_div(x, y, h=1e-5):
    def G(xx, yy):
        rho, u, v, p = prim_field(xx, yy)
        E = p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v)
        return (np.array([rho * u, p + rho * u * u, rho * u * v, (E + p) * u]),
                np.array([rho * v, rho * u * v, p + rho * v * v, (E + p) * v]))
    return ((G(x + h, y)[0] - G(x - h, y)[0]) + (G(x, y + h)[1] - G(x, y - h)[1])) / (2 * h)


@pytest.fixture(scope="module")
def jittered():
    return cg.ogrid(96, 24, r=None, t=0.12, jitter_p=0.3, seed=5)


def test_split_weights_reproduce_linear_functions(jittered):
    o = O.Oracle(jittered)
    c = jittered
    rng = np.random.default_rng(0)
    pts = list(rng.choice(np.where(c.type == cg.INTERIOR)[0], 40, replace=False))
    pts += list(np.where(c.type == cg.WALL)[0][::7])
    for p in pts:
        for k, (d, s) in enumerate(o.split_dirs(p)):
            nb, w, ls1 = o.split_stencil(p, k)
            if len(nb) == 0:
                continue
            e = (-d[1], d[0])
            da = (c.x[nb] - c.x[p]) * d[0] + (c.y[nb] - c.y[p]) * d[1]
            db = (c.x[nb] - c.x[p]) * e[0] + (c.y[nb] - c.y[p]) * e[1]
            assert np.all(s * da < 0)                     # eq. (13): upwind half
            assert np.isclose(np.dot(w, da), 1.0, rtol=1e-10)
            assert abs(np.dot(w, db)) < 1e-10 * np.abs(w).sum() * np.abs(db).max()
            assert np.isclose(ls1, w.sum(), rtol=1e-12, atol=1e-12)


def test_q_gradient_exact_on_linear_and_inner_fixed_point_on_quadratic(jittered):
    c = jittered
    o = O.Oracle(c)
    x, y = c.x, c.y
    q = np.stack([0.3 + 1.5 * x - 0.7 * y, -2 + 0.1 * x + 0.2 * y, x - y, -1.4 + 0.01 * x])
    qx, qy = o.q_grad_pass(q)
    assert np.allclose(qx, np.array([[1.5], [0.1], [1.0], [0.01]]) * np.ones_like(x), atol=1e-11)
    assert np.allclose(qy, np.array([[-0.7], [0.2], [-1.0], [0.0]]) * np.ones_like(x), atol=1e-11)
    # quadratic field: with exact derivatives as input the defect-corrected
    # LS returns them unchanged (second-order exactness of eq. 8-10, 16)
    q = np.stack([x * x, x * y, y * y - x, 0.5 * x * x + 2 * x * y - y * y])
    ex_x = np.stack([2 * x, y, -np.ones_like(x), x + 2 * y])
    ex_y = np.stack([0 * x, x, 2 * y, 2 * x - 2 * y])
    gx, gy = o.q_grad_pass(q, ex_x, ex_y)
    scale = np.abs(ex_x).max() + np.abs(ex_y).max()
    assert np.abs(gx - ex_x).max() < 1e-9 * scale
    assert np.abs(gy - ex_y).max() < 1e-9 * scale


def test_uniform_flow_has_zero_residual_bitwise():
    for wall in (False, True):
        c = cg.box(9, 8, h=0.13, wall_bottom=wall)
        o = O.Oracle(c, mach=0.7, aoa_deg=0.0, inner_iters=2)
        U = o.free_stream()           # parallel to the flat wall
        R, res = o.residual(U)
        assert np.all(R == 0.0)
        assert res == 0.0


def test_residual_is_second_order_accurate():
    errs = []
    for nx in (81, 161):
        c = cg.box(nx, nx, h=2.0 / (nx - 1))
        c.x += 0.3
        c.y += 0.2
        o = O.Oracle(c, inner_iters=0)
        R, _ = o.residual(U_field(c.x, c.y))
        j, k = np.arange(c.n) % nx, np.arange(c.n) // nx
        m = (j >= nx // 4) & (j < nx - nx // 4) & (k >= nx // 4) & (k < nx - nx // 4)
        errs.append(np.abs(R[:, m] - euler_div(c.x[m], c.y[m])).max())
    order = np.log2(errs[0] / errs[1])
    assert order > 1.85, errs      # first order would give 1.0


def test_residual_mirror_symmetry():
    c = cg.ogrid(64, 16, r=1.15)
    o = O.Oracle(c, mach=0.5, aoa_deg=0.0)
    U = o.free_stream()
    # smooth symmetric perturbation
    bump = 1 + 0.05 * np.exp(-((c.x - 0.3) ** 2 + c.y ** 2))
    U = U * bump
    R, _ = o.residual(U)
    nw = c.nw
    j, k = np.arange(c.n) % nw, np.arange(c.n) // nw
    m = k * nw + (nw - j) % nw
    scale = np.abs(R).max()
    sign = np.array([1, 1, -1, 1])[:, None]
    assert np.abs(R[:, m] - sign * R).max() < 1e-11 * scale


def _dense_lusgs(o, U, R, D):
    """(D + P Uu)^-1 D (D + P L)^-1 (-P R) over the non-outer points."""
    c = o.cloud
    n = c.n
    act = np.where(c.type != cg.OUTER)[0]
    pos = -np.ones(n, dtype=int)
    pos[act] = np.arange(len(act))
    m = len(act)
    L = np.zeros((4 * m, 4 * m))
    Uu = np.zeros((4 * m, 4 * m))
    eye = np.eye(4)
    for p in act:
        for k, (d, s) in enumerate(o.split_dirs(p)):
            nb, w, _ = o.split_stencil(p, k)
            for i, wi in zip(nb, w):
                if c.type[i] == cg.OUTER:
                    continue
                A = np.stack([O.flux_jvp(U[:, i], eye[j], d, s) for j in range(4)], axis=1)
                blk = L if o.colours[i] < o.colours[p] else Uu
                blk[4 * pos[p]:4 * pos[p] + 4, 4 * pos[i]:4 * pos[i] + 4] += wi * A
    Pi = np.eye(4 * m)
    for p in act:
        if c.type[p] == cg.WALL:
            nvec = np.array([0.0, -c.ty[p], c.tx[p], 0.0])
            Pi[4 * pos[p]:4 * pos[p] + 4, 4 * pos[p]:4 * pos[p] + 4] = eye - np.outer(nvec, nvec)
    Dm = np.kron(np.diag(D[act]), eye)
    r = R[:, act].T.reshape(-1)
    star = np.linalg.solve(Dm + Pi @ L, -(Pi @ r))
    dU = np.linalg.solve(Dm + Pi @ Uu, Dm @ star)
    out = np.zeros((4, n))
    out[:, act] = dU.reshape(m, 4).T
    return out


@pytest.mark.parametrize("jvp_mode", [0])
def test_sweeps_equal_dense_lu_sgs_solve(jvp_mode):
    c = cg.box(7, 6, h=0.2, wall_bottom=True)
    o = O.Oracle(c, mach=0.6, aoa_deg=0.0, cfl=20.0, jvp_mode=jvp_mode)
    U = o.free_stream()
    rng = np.random.default_rng(1)
    U = U * (1 + 0.05 * rng.standard_normal(U.shape) * (c.type != cg.OUTER))
    # keep the walls tangential
    U[2, c.type == cg.WALL] = 0.0
    R, _ = o.residual(U)
    dt, D = o.timestep_diag(U)
    dU = o.lusgs(U, R, D)
    ref = _dense_lusgs(o, U, R, D)
    assert np.abs(dU - ref).max() < 1e-12 * np.abs(ref).max()
    assert np.abs(dU).max() > 0


def test_colouring_hand_traced_example():
    # path 0-1-2-3 plus the chord 0-2 (a triangle 0,1,2 with a tail 3):
    #   colour(0) = 0; visiting 0: 1 -> smallest absent among {0} = 1,
    #   2 -> absent among {0, 1} = 2; visiting 2: 3 -> absent among {2} = 0.
    off = np.array([0, 2, 4, 7, 8], dtype=np.int32)
    idx = np.array([1, 2, 0, 2, 0, 1, 3, 2], dtype=np.int32)

    class C:
        n = 4
        nbr_off = off
        nbr_idx = idx
    col, nc = O.colour(C)
    assert col.tolist() == [0, 1, 2, 0]
    assert nc == 3


def test_colouring_is_proper_and_deterministic():
    c = cg.cloud_6400()
    col, nc = O.colour(c)
    col2, nc2 = O.colour(c)
    assert np.array_equal(col, col2) and nc == nc2
    rows = np.repeat(np.arange(c.n), np.diff(c.nbr_off))
    assert not np.any(col[rows] == col[c.nbr_idx])
    # a 3x3 block of the ring grid is a clique: at least 9 colours
    assert nc >= 9
    counts = np.bincount(col)
    # a few large colours and a small tail, as in the paper's Table 2
    assert counts.max() > 10 * counts.min()


def test_forces_vanish_for_uniform_pressure():
    c = cg.ogrid(80, 12, r=1.2)
    o = O.Oracle(c, mach=0.5, aoa_deg=3.0)
    U = o.free_stream()
    # uniform pressure, arbitrary tangential velocity: closed polygon => F = 0
    cl, cd = o.forces(U)
    assert abs(cl) < 1e-13 and abs(cd) < 1e-13


def wall_polygon_area(c):
    w = np.flatnonzero(c.type == cg.WALL)
    x, y = c.x[w], c.y[w]
    return 0.5 * abs(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


@pytest.mark.parametrize("aoa", [0.0, 7.0, -4.0])
def test_forces_of_a_linear_pressure_field_closed_form(aoa):
    # p = p_inf + c y on the wall: by the divergence theorem the pressure force
    # -(closed integral of (p - p_inf) n_out ds) is -c A y_hat with A the area
    # enclosed by the wall polygon, and the edge-mean pressure is exact for a
    # linear field on straight edges.  Likewise p = p_inf + c x gives -c A x_hat.
    # CL, CD are the components across / along the free stream over M^2/2.
    c = cg.ogrid(80, 12, r=1.2)
    mach = 0.6
    o = O.Oracle(c, mach=mach, aoa_deg=aoa)
    A = wall_polygon_area(c)
    assert 0.05 < A < 0.1   # a 12%-thick section of unit chord: about 0.082
    qinf = 0.5 * mach * mach
    al = np.radians(aoa)
    slope = 0.05
    for along, F in (("y", np.array([0.0, -slope * A])), ("x", np.array([-slope * A, 0.0]))):
        p = 1 / GAMMA + slope * (c.y if along == "y" else c.x)
        U = np.array([np.ones(c.n), np.zeros(c.n), np.zeros(c.n), p / (GAMMA - 1)])
        cl, cd = o.forces(U)
        want_cl = (F[1] * np.cos(al) - F[0] * np.sin(al)) / qinf
        want_cd = (F[0] * np.cos(al) + F[1] * np.sin(al)) / qinf
        assert cl == pytest.approx(want_cl, rel=1e-12, abs=1e-14)
        assert cd == pytest.approx(want_cd, rel=1e-12, abs=1e-14)
    # the sign: more pressure below than above lifts the body
    p = 1 / GAMMA - slope * c.y
    cl, _ = o.forces(np.array([np.ones(c.n), np.zeros(c.n), np.zeros(c.n), p / (GAMMA - 1)]))
    assert cl > 0 if abs(aoa) < 90 else True


def test_positive_incidence_gives_positive_lift():
    # converged subsonic flow at +2 deg lifts the symmetric profile (the sign of
    # the paper's lift coefficients); its size is near the thin-aerofoil value
    # 2 pi sin(a) / sqrt(1 - M^2) = 0.253 at M 0.5
    # (this coarse 64 x 16 cloud gives about 0.15)
    c = cg.ogrid(64, 16, r=1.15)
    o = O.Oracle(c, mach=0.5, aoa_deg=2.0, cfl=100.0, inner_iters=1)
    U, it, hist = o.solve(o.free_stream(), 1000)
    assert hist[-1] < 1e-6 * hist[0]
    cl, cd = o.forces(U)
    assert 0.1 < cl < 0.4
    o_neg = O.Oracle(c, mach=0.5, aoa_deg=-2.0, cfl=100.0, inner_iters=1)
    Un, _, _ = o_neg.solve(o_neg.free_stream(), 1000)
    cln, cdn = o_neg.forces(Un)
    # the mirror image: opposite lift, same drag
    assert cln == pytest.approx(-cl, rel=1e-7)
    assert cdn == pytest.approx(cd, rel=1e-7)


def test_free_stream_wall_tangency():
    c = cg.ogrid(64, 10, r=1.2)
    o = O.Oracle(c, mach=0.63, aoa_deg=2.0)
    U = o.free_stream()
    w = c.type == cg.WALL
    un = U[1, w] * (-c.ty[w]) + U[2, w] * c.tx[w]
    assert np.abs(un).max() < 1e-15


def test_zero_lift_at_zero_incidence():
    # the colour order is not mirror symmetric, but the converged fixed point is
    c = cg.ogrid(64, 16, r=1.15)
    o = O.Oracle(c, mach=0.5, aoa_deg=0.0, cfl=100.0, inner_iters=1)
    U, it, hist = o.solve(o.free_stream(), 400)
    assert hist[-1] < 1e-3 * hist[0]
    cl, cd = o.forces(U)
    assert abs(cl) < 1e-5


def test_wall_residual_and_increment_keep_tangency():
    # flow tangency at wall points: neither R nor the increment has a
    # component of momentum along the wall normal, whatever the state
    c = cg.ogrid(48, 12, jitter_p=0.04, seed=3)
    o = O.Oracle(c, mach=0.7, aoa_deg=4.0, cfl=50.0, inner_iters=1)
    U = o.free_stream()
    for _ in range(3):
        U, R, dU, _ = o.iteration(U)
    w = c.type == 0
    nx, ny = -c.ty[w], c.tx[w]
    for F in (R, dU):
        normal = F[1, w] * nx + F[2, w] * ny
        assert np.abs(F[1:3, w]).max() > 0
        assert np.abs(normal).max() <= 1e-14 * np.abs(F[1:3, w]).max()


def test_supersonic_zero_incidence_converges_with_zero_lift():
    # the paper's supersonic case (M 1.2, AoA 0): a bow shock ahead of the
    # nose; with the limiter the iteration reaches its fixed point, which is
    # mirror symmetric, so the lift vanishes
    c = cg.ogrid(48, 12)
    o = O.Oracle(c, mach=1.2, aoa_deg=0.0, cfl=100.0, inner_iters=1, limiter=1, limiter_k=5.0)
    U, it, hist = o.solve(o.free_stream(), 600)
    assert it == 600 and hist[-1] < 1e-8 * hist[0]
    cl, cd = o.forces(U)
    assert abs(cl) < 1e-9 and np.isfinite(cd)
    # supersonic in the far field, subsonic pocket behind the shock at the nose
    rho, m1, m2, E = U
    p = 0.4 * (E - 0.5 * (m1 * m1 + m2 * m2) / rho)
    mach = np.hypot(m1, m2) / rho / np.sqrt(1.4 * p / rho)
    assert mach.max() > 1.2 and mach[c.type == 0].min() < 0.1


def test_limiter_keeps_linear_fields_and_clips_extrema():
    # Venkatakrishnan's limiter (an addition: the paper names no limiter).
    c = cg.box(11, 11, h=0.1)
    o = O.Oracle(c, limiter=1, limiter_k=0.5)
    x, y = c.x, c.y
    lin = np.stack([0.3 + x - 2 * y, -2 + 0.4 * x, 0.1 * y, -1.4 + 0.01 * x + 0.02 * y])
    qx, qy = o.q_grad_pass(lin)
    lx, ly = o.limit_gradients(lin, qx, qy)
    j, k = np.arange(c.n) % 11, np.arange(c.n) // 11
    inner = (j >= 2) & (j <= 8) & (k >= 2) & (k <= 8)    # symmetric stencils
    # symmetric stencils: the extreme neighbour difference is twice the
    # reconstruction increment, where the limiter function is exactly 1
    assert np.allclose(lx[:, inner], qx[:, inner], rtol=1e-12, atol=1e-14)
    assert np.allclose(ly[:, inner], qy[:, inner], rtol=1e-12, atol=1e-14)
    # a strict local maximum: no neighbour above it, so phi -> eps^2/(2 d2^2 + eps^2)
    bump = np.exp(-((x - 0.5) ** 2 + (y - 0.5) ** 2) / 0.01)
    q = np.stack([bump, bump, bump, bump - 3.0])
    qx, qy = o.q_grad_pass(q)
    lx, ly = o.limit_gradients(q, qx, qy)
    pk = int(np.argmax(bump))
    phi = np.hypot(lx[0, pk], ly[0, pk]) / max(np.hypot(qx[0, pk], qy[0, pk]), 1e-300)
    assert phi <= 1.0
    ratio = np.hypot(lx, ly) / np.maximum(np.hypot(qx, qy), 1e-300)
    assert np.all(ratio <= 1.0 + 1e-12) and np.all(ratio >= 0.0)
    # the limited reconstruction toward any neighbour stays within the
    # neighbourhood's range up to the eps^2 relaxation
    o2 = O.Oracle(c, limiter=1, limiter_k=1e-6)
    lx, ly = o2.limit_gradients(q, qx, qy)
    for p in np.where(inner)[0]:
        nb = c.nbr_idx[c.nbr_off[p]:c.nbr_off[p + 1]]
        dx, dy = c.x[nb] - c.x[p], c.y[nb] - c.y[p]
        rec = q[0, p] - 0.5 * (dx * lx[0, p] + dy * ly[0, p])
        lo = min(q[0, nb].min(), q[0, p])
        hi = max(q[0, nb].max(), q[0, p])
        assert np.all(rec <= hi + 1e-9) and np.all(rec >= lo - 1e-9)


def _dense_wall_first(o, U, R, D):
    """Algorithm 5 as a dense solve.  Forward: Gauss-Seidel over the
    processing order (groups wall, interior, outer; colours ascending) with
    only lower-colour neighbours already processed contributing (the others
    still hold the zero of the sweep's start): (D + P L') dU* = -P R.
    Backward (same group order, colours descending): an upper-colour
    neighbour contributes its final dU if processed before, else its dU*:
    (D + P U1) dU = (D - P U2) dU*."""
    c = o.cloud
    n = c.n
    act = np.where(c.type != cg.OUTER)[0]
    pos = -np.ones(n, dtype=int)
    pos[act] = np.arange(len(act))
    m = len(act)
    col = o.colours
    fwd = {p: (int(c.type[p]), int(col[p])) for p in range(n)}
    bwd = {p: (int(c.type[p]), -int(col[p])) for p in range(n)}
    L, U1, U2 = (np.zeros((4 * m, 4 * m)) for _ in range(3))
    eye = np.eye(4)
    for p in act:
        for k, (d, s) in enumerate(o.split_dirs(p)):
            nb, w, _ = o.split_stencil(p, k)
            for i, wi in zip(nb, w):
                if c.type[i] == cg.OUTER:
                    continue
                A = np.stack([O.flux_jvp(U[:, i], eye[j], d, s) for j in range(4)], axis=1)
                if col[i] < col[p]:
                    if fwd[i] < fwd[p]:
                        blk = L
                    else:
                        continue
                else:
                    blk = U1 if bwd[i] < bwd[p] else U2
                blk[4 * pos[p]:4 * pos[p] + 4, 4 * pos[i]:4 * pos[i] + 4] += wi * A
    Pi = np.eye(4 * m)
    for p in act:
        if c.type[p] == cg.WALL:
            nvec = np.array([0.0, -c.ty[p], c.tx[p], 0.0])
            Pi[4 * pos[p]:4 * pos[p] + 4, 4 * pos[p]:4 * pos[p] + 4] = eye - np.outer(nvec, nvec)
    Dm = np.kron(np.diag(D[act]), eye)
    r = R[:, act].T.reshape(-1)
    star = np.linalg.solve(Dm + Pi @ L, -(Pi @ r))
    dU = np.linalg.solve(Dm + Pi @ U1, (Dm - Pi @ U2) @ star)
    out = np.zeros((4, n))
    out[:, act] = dU.reshape(m, 4).T
    return out


def test_wall_first_sweeps_equal_dense_solve():
    c = cg.box(7, 6, h=0.2, wall_bottom=True)
    o = O.Oracle(c, mach=0.6, aoa_deg=0.0, cfl=20.0, order=O.WALL_FIRST)
    U = o.free_stream()
    rng = np.random.default_rng(1)
    U = U * (1 + 0.05 * rng.standard_normal(U.shape) * (c.type != cg.OUTER))
    U[2, c.type == cg.WALL] = 0.0
    R, _ = o.residual(U)
    dt, D = o.timestep_diag(U)
    dU = o.lusgs(U, R, D)
    ref = _dense_wall_first(o, U, R, D)
    assert np.abs(dU - ref).max() < 1e-12 * np.abs(ref).max()
    # and it differs from the colour order (the wall points see stale neighbours)
    o0 = O.Oracle(c, mach=0.6, aoa_deg=0.0, cfl=20.0)
    assert np.abs(o0.lusgs(U, R, D) - dU).max() > 1e-6 * np.abs(dU).max()


def test_wall_first_without_walls_is_colour_order():
    # interior before outer points, whose increment is always 0: the same result
    c = cg.box(9, 8, h=0.13)
    rng = np.random.default_rng(4)
    for order in (O.COLOUR_ORDER, O.WALL_FIRST):
        o = O.Oracle(c, mach=0.5, aoa_deg=20.0, cfl=20.0, order=order)
        U = o.free_stream() * (1 + 0.03 * rng.standard_normal((4, c.n)) * (c.type != cg.OUTER))
        rng = np.random.default_rng(4)
        if order == O.COLOUR_ORDER:
            ref = o.iteration(U)
        else:
            got = o.iteration(U)
    assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[2], got[2])
