"""Pins of the oracle's van der Waals force (Sec. 2.2, Eqs. (17)-(23)).

  * Korteweg identity: at uniform T the divergence of the gradient part of the
    pressure tensor (Eq. (19)) is -K rho grad(lap rho).
  * The temperature term of Eq. (19) equals -rho T grad rho . grad(M/T) formed by
    differentiating the field M/T itself.
  * Total energy (Eq. (17)) is conserved by the continuous dynamics (Eq. (14)); with
    exact wavenumbers on band-limited fields the oracle's first-order energy rate
    vanishes to round-off, which fixes every term of C (Eq. (22)) and C_q (Eq. (23)).
  * A planar and a diagonal interface in van der Waals equilibrium (the interface
    of Eqs. (51)-(53)) are in mechanical balance: the force cancels the ideal-gas
    pressure gradient, which fixes P^w, S and Lambda.
  * Special case a = b = K = q = 0 (the ideal-gas model of Sec. 2.1): I = 0 exactly.
"""
import math

import numpy as np
import pytest

from oracle import fftlb_oracle as O
from oracle import thermo


def _band_limited(n, rng, amp, modes=2, mean=0.0):
    x = 2 * np.pi * np.arange(n)[None, :] / n
    y = 2 * np.pi * np.arange(n)[:, None] / n
    out = np.full((n, n), mean)
    for kx in range(-modes, modes + 1):
        for ky in range(-modes, modes + 1):
            if kx == 0 and ky == 0:
                continue
            out += amp * rng.normal() * np.cos(kx * x + ky * y + rng.uniform(0, 2 * np.pi)) / (2 * modes + 1)
    return out


def test_korteweg_identity():
    n = 48
    rng = np.random.default_rng(11)
    p = O.Params(dx=1 / 48, dy=1 / 48, K=0.03, H=0.0, m=0, a=1.0, b=0.3)
    D = O.Deriv(n, n, p)
    rho = _band_limited(n, rng, 0.3, mean=1.0)
    u = _band_limited(n, rng, 0.1)
    T = np.full((n, n), 0.9)
    fc = O.force_coefficients(rho, u, 0.5 * u, T, p, D)
    div_x = D.x(fc.Lxx) + D.y(fc.Lxy)
    div_y = D.x(fc.Lxy) + D.y(fc.Lyy)
    lap = D.x(D.x(rho)) + D.y(D.y(rho))
    ref_x = -p.K * rho * D.x(lap)
    ref_y = -p.K * rho * D.y(lap)
    scale = np.abs(ref_x).max()
    assert scale > 1e-2
    np.testing.assert_allclose(div_x, ref_x, atol=1e-10 * scale)
    np.testing.assert_allclose(div_y, ref_y, atol=1e-10 * scale)


@pytest.mark.parametrize("H", [0.0, 0.02])
def test_lambda_temperature_term(H):
    n = 32
    rng = np.random.default_rng(12)
    p = O.Params(dx=1 / 32, dy=1 / 32, K=0.02, H=H, m=0)
    D = O.Deriv(n, n, p)
    rho = _band_limited(n, rng, 0.2, mean=1.0)
    T = _band_limited(n, rng, 0.1, mean=1.0)
    z = np.zeros((n, n))
    fc = O.force_coefficients(rho, z, z, T, p, D)
    M = p.K + p.H * T
    lap = D.x(D.x(rho)) + D.y(D.y(rho))
    rx, ry = D.x(rho), D.y(rho)
    MT = M / T
    temp_term = -rho * T * (rx * D.x(MT) + ry * D.y(MT))
    ref_xx = M * rx * rx + temp_term - M * (rho * lap + 0.5 * (rx * rx + ry * ry))
    # the band-limited rule for M/T holds to the spectral accuracy of 1/T
    np.testing.assert_allclose(fc.Lxx, ref_xx, atol=1e-9 * np.abs(ref_xx).max())
    np.testing.assert_allclose(fc.Lxy, M * rx * ry, atol=1e-12 * np.abs(fc.Lxy).max())


def _energy(f, p, D):
    rho, ux, uy, T = O.moments(f)
    e = O.total_energy_density(rho, ux, uy, T, D.x(rho), D.y(rho), p)
    return e.sum() * p.dx * p.dy


@pytest.mark.parametrize("zeta,q,K", [(0.0, -0.004, 0.02), (0.01, 0.03, 0.05), (0.0, 0.0, 0.0)])
def test_total_energy_rate_vanishes(zeta, q, K):
    """With f = f^eq the collision is idle and dE/dt comes from convection and the force only.
    Eq. (14) makes it zero in the continuum; here it is evaluated by a central difference in the
    step direction, so no time-discretisation error enters."""
    n = 64
    rng = np.random.default_rng(13)
    p = O.Params(dx=1 / 64, dy=1 / 64, K=K, H=0.0, zeta=zeta, q=q, m=0, a=1.2, b=0.3, dt=1e-6)
    D = O.Deriv(n, n, p)
    rho = _band_limited(n, rng, 0.04, mean=1.0)
    ux = _band_limited(n, rng, 0.05)
    uy = _band_limited(n, rng, 0.05)
    T = _band_limited(n, rng, 0.03, mean=1.0)
    f0 = O.feq(rho, ux, uy, T)
    parts = O.step_parts(f0, p)
    R = (parts.f_next - f0) / p.dt
    h = 1e-5
    rate = (_energy(f0 + h * R, p, D) - _energy(f0 - h * R, p, D)) / (2 * h)
    # reference size: the work of the nonideal pressure alone
    fc = parts.force
    scale = abs((p.a * rho * rho * fc.theta).sum() * p.dx * p.dy) + abs((fc.C * rho * T * T).sum() * p.dx * p.dy)
    assert scale > 1e-4
    assert abs(rate) < 1e-8 * scale, (rate, scale)


def test_energy_rate_detects_a_dropped_term():
    """Sanity check of the energy pin: removing the -rho grad rho . grad theta term of C
    breaks the balance by far more than the tolerance used above."""
    n = 64
    rng = np.random.default_rng(13)
    p = O.Params(dx=1 / 64, dy=1 / 64, K=0.02, H=0.0, zeta=0.0, q=-0.004, m=0, a=1.2, b=0.3, dt=1e-6)
    D = O.Deriv(n, n, p)
    rho = _band_limited(n, rng, 0.04, mean=1.0)
    ux = _band_limited(n, rng, 0.05)
    uy = _band_limited(n, rng, 0.05)
    T = _band_limited(n, rng, 0.03, mean=1.0)
    f0 = O.feq(rho, ux, uy, T)
    good = O.force_coefficients(rho, ux, uy, T, p, D)
    th = good.theta
    extra = -p.K * rho * (good.rx * D.x(th) + good.ry * D.y(th)) / (2 * rho * T * T)
    # work done by the term alone (its kinetic-energy moment is -2 rho T^2 C_term)
    work = np.abs((-2 * rho * T * T * extra).sum() * p.dx * p.dy)
    scale = abs((p.a * rho * rho * th).sum() * p.dx * p.dy)
    assert work > 1e-5 * scale


def _equilibrium_slab(ny, nx, p, T, diagonal=False):
    """Periodic slab between two van der Waals equilibrium interfaces, normal along x (or along
    the diagonal), built from the planar profile.  The interfaces are far enough apart that
    the profile's tails have decayed below 1e-13 where they meet."""
    L = nx * p.dx
    x = np.arange(nx) * p.dx
    y = np.arange(ny) * p.dy
    if diagonal:
        period = L / math.sqrt(2.0)        # rho(x, y) = P((x + y)/sqrt 2), period L/sqrt 2 along the normal
        s = (x[None, :] + y[:, None]) / math.sqrt(2.0)
    else:
        period = L
        s = np.broadcast_to(x[None, :], (ny, nx))
    s = np.mod(s, period)
    left, right = period / 4, 3 * period / 4
    d = np.where(s < period / 2, s - left, right - s)   # > 0 in the liquid between the interfaces
    return thermo.planar_profile(d, T, p.a, p.b, p.K)


@pytest.mark.parametrize("diagonal", [False, True])
def test_equilibrium_interface_feels_no_force(diagonal):
    ny, nx = (512, 512) if diagonal else (4, 512)
    T = 0.95
    p = O.Params(dx=1 / 256, dy=1 / 256, K=2e-5, H=0.0, q=-0.004, m=0, a=9 / 8, b=1 / 3)
    rho = _equilibrium_slab(ny, nx, p, T, diagonal)
    z = np.zeros((ny, nx))
    D = O.Deriv(ny, nx, p)
    fc = O.force_coefficients(rho, z, z, np.full((ny, nx), T), p, D)
    drive = np.abs(D.x(fc.Pw)).max()          # the pressure gradient the interface has to balance
    assert drive > 0.1
    # Streaming of f^eq carries the ideal pressure rho T (its second moment, Eq. (3));
    # the force adds -rho T B (Eq. (11)).  At equilibrium the two cancel:
    # d_a(rho T) + rho T B_a = d_b(P^w delta_ab + Lambda_ab) = 0.
    net_x = D.x(rho * T) + fc.Bx * rho * T
    net_y = D.y(rho * T) + fc.By * rho * T
    assert np.hypot(net_x, net_y).max() < 1e-8 * drive, (np.hypot(net_x, net_y).max(), drive)
    # the balance needs the gradient terms: Lambda's divergence is of the same size as the drive
    assert np.abs(D.x(fc.Lxx) + D.y(fc.Lxy)).max() > 0.1 * drive


def test_ideal_gas_has_no_force():
    n = 32
    rng = np.random.default_rng(14)
    p = O.Params(dx=1 / 32, dy=1 / 32, K=0.0, H=0.0, zeta=0.0, q=0.0, a=0.0, b=0.0, m=4)
    rho = _band_limited(n, rng, 0.2, mean=1.0, modes=5)
    ux, uy = _band_limited(n, rng, 0.1, modes=5), _band_limited(n, rng, 0.1, modes=5)
    T = _band_limited(n, rng, 0.1, mean=1.0, modes=5)
    fc = O.force_coefficients(rho, ux, uy, T, p, O.Deriv(n, n, p))
    I = O.force_term(O.feq(rho, ux, uy, T), ux, uy, fc)
    assert np.all(I == 0.0)


def test_conservative_divergence_matches_product_rule():
    """Reading R3 (divergence of the product field) agrees with the expanded product rule on
    band-limited fields with exact wavenumbers."""
    n = 32
    rng = np.random.default_rng(15)
    p = O.Params(dx=1 / 32, dy=1 / 32, q=0.05, m=0, K=0.0)
    D = O.Deriv(n, n, p)
    rho = _band_limited(n, rng, 0.2, mean=1.0)
    T = _band_limited(n, rng, 0.1, mean=1.0)
    z = np.zeros((n, n))
    fc = O.force_coefficients(rho, z, z, T, p, D)
    Tx, Ty = D.x(T), D.y(T)
    rT = rho * T
    expanded = 2 * p.q * (rT * (D.x(Tx) + D.y(Ty)) + D.x(rT) * Tx + D.y(rT) * Ty)
    np.testing.assert_allclose(fc.Cq * 2 * rho * T * T, expanded, atol=1e-11 * np.abs(expanded).max())
