"""Pins of the oracle's kinetic split fluxes and their Jacobian-vector products.

The split fluxes are the half-range moments <Psi, v_d F> of the Maxwellian of
eq. (3)-(4) (Section 2, CIR splitting eq. 5 -> KFVS eq. 6).  The paper prints
no closed form, so the oracle's closed form is pinned here against direct
numerical quadrature of those moments, against G+ + G- = G (eq. 2), and
against the limits S -> +-inf.  The exact Jacobian-vector products are pinned
against central differences of the flux and, summed over the two halves,
against the complex-step derivative of the unsplit flux of eq. (2).
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O

GAMMA = 1.4


def U_of(rho, u1, u2, p, g=GAMMA):
    return np.array([rho, rho * u1, rho * u2, p / (g - 1) + 0.5 * rho * (u1 * u1 + u2 * u2)])


def unsplit_flux(U, d, g=GAMMA):
    """Eq. (2): Gx, Gy combined along unit direction d."""
    rho, m1, m2, E = U
    u1, u2 = m1 / rho, m2 / rho
    p = (g - 1) * (E - 0.5 * rho * (u1 * u1 + u2 * u2))
    ud = u1 * d[0] + u2 * d[1]
    return np.array([rho * ud, p * d[0] + m1 * ud, p * d[1] + m2 * ud, (E + p) * ud])


def unsplit_jvp(U, dU, d, g=GAMMA, h=1e-30):
    """Unsplit flux Jacobian times dU along d by complex-step differentiation
    of eq. (2): the flux is a rational function of U, so
    Im F(U + i h dU) / h is its directional derivative to rounding."""
    return np.imag(unsplit_flux(np.asarray(U, complex) + 1j * h * np.asarray(dU, complex),
                                d, g)) / h


def quad_split_flux(rho, u1, u2, p, d, s, g=GAMMA):
    """<Psi, v_d F> over the half space s*v_d > 0 by numerical quadrature.

    F = rho/I0 * beta/pi * exp(-beta |v - u|^2 - I/I0) (eq. 4); integrating
    over I >= 0 leaves the 2D Maxwellian with mean internal energy I0, where
    rho E = rho (|u|^2/2 + 1/(2 beta) + I0) fixes I0 = (2 - g)/(2 beta (g - 1)).
    """
    beta = rho / (2 * p)
    I0 = (2 - g) / (2 * beta * (g - 1))
    e = (-d[1], d[0])
    ud = u1 * d[0] + u2 * d[1]
    ut = u1 * e[0] + u2 * e[1]
    # integrate over the peculiar velocities c = v - u in the (d, e) frame
    width = 12.0 / math.sqrt(beta)

    def f(ct, cd, comp):
        vd = ud + cd
        vt = ut + ct
        vx = vd * d[0] + vt * e[0]
        vy = vd * d[1] + vt * e[1]
        w = rho * beta / math.pi * math.exp(-beta * (cd * cd + ct * ct)) * vd
        psi = (1.0, vx, vy, I0 + 0.5 * (vx * vx + vy * vy))[comp]
        return w * psi

    out = []
    for comp in range(4):
        if s > 0:
            lo, hi = -ud, max(-ud, 0.0) + width
            lo = max(lo, -width)
        else:
            lo, hi = min(-ud, 0.0) - width, -ud
            hi = min(hi, width)
        val, _ = integrate.dblquad(f, lo, hi, -width, width, args=(comp,), epsabs=1e-13,
                                   epsrel=1e-12)
        out.append(val)
    return np.array(out)


STATES = [
    (1.0, 0.3, 0.1, 1 / GAMMA),
    (0.7, -0.9, 0.4, 0.5),
    (1.3, 1.6, -0.2, 1.2),
    (0.9, 0.0, 0.0, 0.6),
]
DIRS = [(1.0, 0.0), (0.0, 1.0), (0.6, 0.8), (-0.28, 0.96)]


@pytest.mark.parametrize("state", STATES)
@pytest.mark.parametrize("d", DIRS[:3])
@pytest.mark.parametrize("s", [1, -1])
def test_split_flux_matches_moment_quadrature(state, d, s):
    G = O.split_flux(U_of(*state), d, s)
    Q = quad_split_flux(*state, d, s)
    assert np.allclose(G, Q, rtol=1e-9, atol=1e-11), (G, Q)


@pytest.mark.parametrize("state", STATES)
@pytest.mark.parametrize("d", DIRS)
def test_split_fluxes_sum_to_euler_flux(state, d):
    U = U_of(*state)
    G = O.split_flux(U, d, 1) + O.split_flux(U, d, -1)
    assert np.allclose(G, unsplit_flux(U, d), rtol=2e-15, atol=2e-15)


def test_split_flux_limits():
    # S = u sqrt(beta) -> +inf: all molecules move along +d
    U = U_of(1.0, 12.0, 0.3, 1 / GAMMA)
    d = (1.0, 0.0)
    assert np.allclose(O.split_flux(U, d, 1), unsplit_flux(U, d), rtol=1e-14, atol=1e-14)
    assert np.allclose(O.split_flux(U, d, -1), 0.0, atol=1e-14)
    # at rest: mass fluxes rho B and -rho B with B = 1/(2 sqrt(pi beta))
    rho, p = 1.2, 0.8
    beta = rho / (2 * p)
    U = U_of(rho, 0.0, 0.0, p)
    Gp, Gm = O.split_flux(U, d, 1), O.split_flux(U, d, -1)
    B = 1 / (2 * math.sqrt(math.pi * beta))
    assert math.isclose(Gp[0], rho * B, rel_tol=1e-15)
    assert math.isclose(Gm[0], -rho * B, rel_tol=1e-15)
    # momentum: half the pressure each way
    assert math.isclose(Gp[1], 0.5 * p, rel_tol=1e-15)


@pytest.mark.parametrize("state", STATES)
@pytest.mark.parametrize("d", DIRS)
@pytest.mark.parametrize("s", [1, -1])
def test_exact_jvp_is_flux_derivative(state, d, s):
    U = U_of(*state)
    rng = np.random.default_rng(7)
    dU = rng.standard_normal(4) * np.array([0.1, 0.1, 0.1, 0.3])
    J = O.flux_jvp(U, dU, d, s, jvp_mode=0)
    # 4th-order central difference of the oracle's own flux
    h = 1e-3
    f = lambda t: O.split_flux(U + t * dU, d, s)
    fd = (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)
    assert np.allclose(J, fd, rtol=1e-9, atol=1e-10), (J, fd)


@pytest.mark.parametrize("state", STATES)
@pytest.mark.parametrize("d", DIRS)
def test_split_jvps_sum_to_unsplit_jacobian_product(state, d):
    U = U_of(*state)
    rng = np.random.default_rng(11)
    for _ in range(4):
        dU = rng.standard_normal(4)
        J = O.flux_jvp(U, dU, d, 1) + O.flux_jvp(U, dU, d, -1)
        ref = unsplit_jvp(U, dU, d)
        assert np.allclose(J, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max()), (J, ref)


def test_flux_difference_converges_quadratically_to_tangent():
    U = U_of(1.1, 0.45, -0.2, 0.8)
    d, s = (0.6, 0.8), 1
    dU = np.array([0.2, -0.1, 0.3, 0.5])
    J = O.flux_jvp(U, dU, d, s, jvp_mode=0)
    errs = []
    for eps in [1e-2, 5e-3, 2.5e-3]:
        Jfd = O.flux_jvp(U, eps * dU, d, s, jvp_mode=1) / eps
        errs.append(np.abs(Jfd - J).max())
    # eq. (28) is the first-order Taylor term: the error of FD/eps is O(eps)
    assert errs[0] / errs[1] == pytest.approx(2.0, rel=0.05)
    assert errs[1] / errs[2] == pytest.approx(2.0, rel=0.05)
    assert errs[2] < 1e-3 * np.abs(J).max()


def test_q_variables_round_trip():
    rng = np.random.default_rng(3)
    n = 50
    rho = rng.uniform(0.3, 2.0, n)
    u1 = rng.uniform(-1.5, 1.5, n)
    u2 = rng.uniform(-1.5, 1.5, n)
    p = rng.uniform(0.2, 2.0, n)
    U = U_of(rho, u1, u2, p)
    q = O.q_from_U(U)
    beta = rho / (2 * p)
    # eq. (14) componentwise
    assert np.allclose(q[1], 2 * beta * u1, rtol=1e-15)
    assert np.allclose(q[3], -2 * beta, rtol=1e-15)
    assert np.allclose(q[0], np.log(rho) + np.log(beta) / (GAMMA - 1) - beta * (u1 ** 2 + u2 ** 2),
                       rtol=1e-14, atol=1e-14)
    U2 = O.U_from_q(q)
    assert np.allclose(U2, U, rtol=5e-15, atol=5e-15)
