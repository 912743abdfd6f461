"""Pins of the exact ideal-gas Riemann solution (oracle/riemann.py) used for the modified
Sod tube: the textbook Sod star state (gamma = 1.4), and, for the paper's gamma = 2 tube, the
Rankine-Hugoniot conditions across the computed shock, the isentrope and Riemann invariant
across the computed rarefaction, and continuity of p and u across the contact."""
import math

import numpy as np
import pytest

from oracle import riemann as R

SOD = (1.0, 0.0, 1.0, 0.125, 0.0, 0.1)


def test_textbook_sod_star_state():
    # Sod's problem, gamma = 1.4: p* = 0.30313, u* = 0.92745, rho*_L = 0.42632, rho*_R = 0.26557
    p, u = R.star_state(*SOD, 1.4)
    rl, rr = R.star_densities(1.0, 1.0, 0.125, 0.1, p, 1.4)
    assert p == pytest.approx(0.30313, abs=5e-6) and u == pytest.approx(0.92745, abs=5e-6)
    assert rl == pytest.approx(0.42632, abs=5e-6) and rr == pytest.approx(0.26557, abs=5e-6)


# The paper's modified tube: (rho, u, T)_L = (1, 0, 1), (rho, u, T)_R = (0.125, 0, 0.5), p = rho T
TUBE = (1.0, 0.0, 1.0, 0.125, 0.0, 0.0625)
G = 2.0


def _fan(xi):
    return R.sample(np.asarray(xi), *TUBE, G)


def test_shock_satisfies_rankine_hugoniot():
    p_s, u_s = R.star_state(*TUBE, G)
    assert p_s > TUBE[5]                                   # a right-moving shock
    xi = np.linspace(u_s + 1e-9, 4.0, 200001)
    rho, u, p = _fan(xi)
    k = np.argmax(rho < 0.5 * (rho[0] + TUBE[3]))          # the jump
    S = 0.5 * (xi[k - 1] + xi[k])
    (r1, u1, p1), (r2, u2, p2) = (rho[k - 1], u[k - 1], p[k - 1]), (rho[k], u[k], p[k])
    e = lambda r, uu, pp: pp / (G - 1.0) + 0.5 * r * uu * uu     # total energy per volume
    assert r1 * (u1 - S) == pytest.approx(r2 * (u2 - S), rel=1e-4)
    assert r1 * u1 * (u1 - S) + p1 == pytest.approx(r2 * u2 * (u2 - S) + p2, rel=1e-4)
    assert (e(r1, u1, p1) + p1) * u1 - S * e(r1, u1, p1) == pytest.approx((e(r2, u2, p2) + p2) * u2 - S * e(r2, u2, p2),
                                                                          rel=1e-4)


def test_rarefaction_is_isentropic_with_constant_riemann_invariant():
    p_s, u_s = R.star_state(*TUBE, G)
    c_l = math.sqrt(G * TUBE[2] / TUBE[0])
    xi = np.linspace(-c_l - 0.5, u_s - 1e-9, 5001)
    rho, u, p = _fan(xi)
    s = p / rho ** G
    c = np.sqrt(G * p / rho)
    assert np.abs(s / s[0] - 1.0).max() < 1e-12
    J = u + 2.0 * c / (G - 1.0)
    assert np.abs(J - J[0]).max() < 1e-12
    assert rho.max() == pytest.approx(1.0) and rho.min() < 0.6


def test_contact_carries_pressure_and_velocity():
    p_s, u_s = R.star_state(*TUBE, G)
    rho, u, p = _fan([u_s - 1e-9, u_s + 1e-9])
    assert p[0] == pytest.approx(p[1], rel=1e-14) and u[0] == pytest.approx(u[1], rel=1e-14)
    assert rho[0] > rho[1]                                  # the density jumps
