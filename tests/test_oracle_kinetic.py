"""Pins of the oracle's kinetic model (Sec. 2.1): velocities, weights, equilibrium, force moments.

Every check compares the oracle with something other than itself: numbers the
paper prints, moments of the continuous Maxwellian computed by quadrature, the
Taylor series of the Maxwellian, or exact moment identities.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import fftlb_oracle as O

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_velocity_set_matches_paper():
    v = O.velocities()
    assert v.shape == (33, 2)
    assert np.all(v[0] == 0.0)
    speeds = GOLDEN["speeds"]["value"]
    for k in range(4):
        grp = v[1 + 8 * k: 9 + 8 * k]
        np.testing.assert_allclose(np.hypot(grp[:, 0], grp[:, 1]), speeds[k], rtol=0, atol=1e-15)
        ang = np.mod(np.arctan2(grp[:, 1], grp[:, 0]), 2 * np.pi)
        np.testing.assert_allclose(ang, np.arange(8) * np.pi / 4, atol=1e-14)
    # axis-aligned velocities have exact zero components
    assert v[3, 0] == 0.0 and v[1, 1] == 0.0


def _maxwellian_radial_moment(n, T):
    """int |v|^(2n) exp(-|v|^2/2T)/(2 pi T) d^2v by quadrature (polar coordinates)."""
    val, _ = integrate.quad(lambda r: r ** (2 * n) * math.exp(-r * r / (2 * T)) * r / T, 0, np.inf,
                            epsabs=0, epsrel=1e-13)
    return val


@pytest.mark.parametrize("T", [0.5, 0.85, 0.95, 1.0, 1.185185, 1.333333, 1.452])
def test_weights_reproduce_maxwellian_moments(T):
    F0, F = O.weights(T)
    s = np.array(O.SPEEDS) ** 2
    assert abs(F0 + 8 * sum(F) - 1.0) < 1e-15
    for n in range(1, 5):
        disc = 8 * sum(F[k] * s[k] ** n for k in range(4))
        assert disc == pytest.approx(_maxwellian_radial_moment(n, T), rel=1e-12)


def test_weights_table_values():
    # weights at T = 1 spot-checked against an independent exact rational evaluation
    from fractions import Fraction as Fr
    s = [Fr(1), Fr(361, 100), Fr(841, 100), Fr(1849, 100)]
    T = Fr(1)
    F0, F = O.weights(1.0)
    for k in range(4):
        o = [s[(k + l) % 4] for l in (1, 2, 3)]
        num = 48 * T**4 - 6 * sum(o) * T**3 + (o[0] * o[1] + o[1] * o[2] + o[2] * o[0]) * T**2 - o[0] * o[1] * o[2] * T / 4
        den = s[k] * (s[k] - o[0]) * (s[k] - o[1]) * (s[k] - o[2])
        assert F[k] == pytest.approx(float(num / den), rel=1e-14)
        assert F[k] > 0


def _rand_state(rng, shape=(5, 7), umax=0.3):
    rho = rng.uniform(0.2, 1.6, shape)
    ang = rng.uniform(0, 2 * np.pi, shape)
    mag = rng.uniform(0, umax, shape)
    return rho, mag * np.cos(ang), mag * np.sin(ang), rng.uniform(0.6, 1.5, shape)


def test_feq_is_fourth_order_taylor_of_maxwellian():
    """Eq. (3): rho F_k exp((2 u.v - u^2)/2T) expanded to 4th order in u; the remainder is O(|u|^5)."""
    rng = np.random.default_rng(1)
    rho, ux, uy, T = _rand_state(rng, (3, 4), umax=1.0)
    v = O.velocities()
    F0, F = O.weights(T)
    Fk = np.stack([F0] + [F[(q - 1) // 8] for q in range(1, 33)])
    errs = []
    for lam in (0.02, 0.01):
        fe = O.feq(rho, lam * ux, lam * uy, T)
        vu = lam * (v[:, 0, None, None] * ux + v[:, 1, None, None] * uy)
        u2 = lam * lam * (ux * ux + uy * uy)
        exact = rho * Fk * np.exp((2 * vu - u2) / (2 * T))
        errs.append(np.abs(fe - exact).max())
    ratio = errs[0] / errs[1]
    assert 28 < ratio < 36, ratio          # fifth order: halving u divides the error by 32


def test_feq_moments_are_exact():
    """Moments of Eq. (3) up to fourth order equal those of the Maxwellian (Eqs. (7)-(9))."""
    rng = np.random.default_rng(2)
    rho, ux, uy, T = _rand_state(rng)
    fe = O.feq(rho, ux, uy, T)
    v = O.velocities()
    cx = v[:, 0, None, None] - ux
    cy = v[:, 1, None, None] - uy
    c2 = cx * cx + cy * cy
    tol = 1e-13
    np.testing.assert_allclose(fe.sum(0), rho, rtol=tol)
    np.testing.assert_allclose((v[:, 0, None, None] * fe).sum(0), rho * ux, atol=tol)
    np.testing.assert_allclose((v[:, 1, None, None] * fe).sum(0), rho * uy, atol=tol)
    np.testing.assert_allclose((0.5 * c2 * fe).sum(0), rho * T, rtol=tol)
    np.testing.assert_allclose((cx * cx * fe).sum(0), rho * T, rtol=tol)
    np.testing.assert_allclose((cy * cy * fe).sum(0), rho * T, rtol=tol)
    np.testing.assert_allclose((cx * cy * fe).sum(0), 0 * rho, atol=tol)
    np.testing.assert_allclose((cx * c2 * fe).sum(0), 0 * rho, atol=10 * tol)
    np.testing.assert_allclose((cy * c2 * fe).sum(0), 0 * rho, atol=10 * tol)
    np.testing.assert_allclose((c2 * c2 * fe).sum(0), 8 * rho * T * T, rtol=10 * tol)


def test_moments_recover_fields():
    rng = np.random.default_rng(3)
    rho, ux, uy, T = _rand_state(rng)
    r2, ux2, uy2, T2 = O.moments(O.feq(rho, ux, uy, T))
    np.testing.assert_allclose(r2, rho, rtol=1e-14)
    np.testing.assert_allclose(ux2, ux, atol=1e-14)
    np.testing.assert_allclose(uy2, uy, atol=1e-14)
    np.testing.assert_allclose(T2, T, rtol=1e-13)


def test_force_term_moments():
    """Eq. (11) with A = -2(C + C_q)T (Eq. (20)) adds no mass, momentum -rho T B and
    kinetic energy -2 rho T^2 (C + C_q): the constraints the coefficients are built on."""
    rng = np.random.default_rng(4)
    rho, ux, uy, T = _rand_state(rng)
    shape = rho.shape
    C, Cq = rng.normal(size=shape), rng.normal(size=shape)
    Bx, By = rng.normal(size=shape), rng.normal(size=shape)
    fc = O.Force(A=-2 * (C + Cq) * T, Bx=Bx, By=By, C=C, Cq=Cq, rx=None, ry=None, lap=None,
                 theta=None, Pw=None, Lxx=None, Lxy=None, Lyy=None)
    fe = O.feq(rho, ux, uy, T)
    I = O.force_term(fe, ux, uy, fc)
    v = O.velocities()
    cx = v[:, 0, None, None] - ux
    cy = v[:, 1, None, None] - uy
    scale = np.abs(I).max()
    np.testing.assert_allclose(I.sum(0), 0 * rho, atol=1e-14 * scale * 33)
    np.testing.assert_allclose((cx * I).sum(0), -rho * T * Bx, atol=1e-13 * scale * 33)
    np.testing.assert_allclose((cy * I).sum(0), -rho * T * By, atol=1e-13 * scale * 33)
    np.testing.assert_allclose((0.5 * (cx * cx + cy * cy) * I).sum(0), -2 * rho * T * T * (C + Cq),
                               atol=1e-12 * scale * 33)
