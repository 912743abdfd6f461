"""Pins of the oracle's finite-difference convection schemes (Sec. 3.1: Lax-Wendroff,
Eq. (ML-); MLW1 = LW + R3, Eq. (R3); MLW2 = LW + R3 + R4, Eq. (R4=)) against facts fixed
outside their formulas:

  * at CFL number c = +-1 every scheme moves a profile by exactly one node (the R3 and R4
    terms carry the factor 1 - c^2, and LW is then the exact shift);
  * the updates of all schemes conserve the sum over the periodic grid (mass);
  * on a smooth mode the R3 term is dt times the dispersion term of the modified equation
    (Eq. (MPDE), first term: v (1 - c^2)/6 dr^2 d^3f/dr^3) and the R4 term dt times its
    dissipation term (second term: v c (1 - c^2)/8 dr^3 d^4f/dr^4), to leading order in
    the wavenumber;
  * LW's one-step error against exact translation is the dispersion term of Eq. (MPDE)
    (third order in k dr), and adding R3 removes it (MLW1's error is of fourth order);
  * c -> 0: the LW update over c tends to the second-order central difference, MLW1's and
    MLW2's to the fourth-order one (-g[J+2] + 8 g[J+1] - 8 g[J-1] + g[J-2]) / 12;
  * in a full step, populations moving along y only are changed only by the y stencil.
"""
import math

import numpy as np
import pytest

from oracle import fftlb_oracle as O

SCHEMES = (O.LAX_WENDROFF, O.MLW1, O.MLW2)


def _profile(n=64, seed=3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("c,shift", [(1.0, 1), (-1.0, -1)])
def test_unit_cfl_is_an_exact_shift(scheme, c, shift):
    g = _profile()
    out = g + O.fd_convection_update(g, c, 0, scheme)
    # c = v dt / dx = 1: the profile moves one node in +x, g^{n+1}[J] = g[J - 1]
    assert np.allclose(out, np.roll(g, shift), rtol=0, atol=1e-13)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_update_conserves_the_sum(scheme):
    g = _profile(48, seed=5).reshape(6, 8)
    for axis in (0, 1):
        du = O.fd_convection_update(g, 0.37, axis, scheme)
        assert abs(du.sum()) < 1e-13


def _mode(n, m):
    J = np.arange(n)
    theta = 2.0 * np.pi * m / n
    return J, theta


def test_r3_and_r4_are_the_modified_equation_terms():
    # g = cos(k x) with x = J dr: d^3g/dx^3 = k^3 sin(kx), d^4g/dx^4 = k^4 cos(kx).
    # Eq. (MPDE): the terms added are dt v (1 - c^2)/6 dr^2 g''' and dt v c (1 - c^2)/8 dr^3 g''''.
    n, dr, dt, v = 4096, 1.0 / 256.0, 1e-3, 0.9
    c = v * dt / dr
    for m in (4, 8):
        J, theta = _mode(n, m)
        k = theta / dr
        g = np.cos(theta * J)
        r3 = O.fd_convection_update(g, c, 0, O.MLW1) - O.fd_convection_update(g, c, 0, O.LAX_WENDROFF)
        r4 = O.fd_convection_update(g, c, 0, O.MLW2) - O.fd_convection_update(g, c, 0, O.MLW1)
        want3 = dt * v * (1 - c * c) / 6.0 * dr ** 2 * k ** 3 * np.sin(theta * J)
        want4 = dt * v * c * (1 - c * c) / 8.0 * dr ** 3 * k ** 4 * np.cos(theta * J)
        # relative difference O(theta^2)
        assert np.abs(r3 - want3).max() <= 0.5 * theta ** 2 * np.abs(want3).max()
        assert np.abs(r4 - want4).max() <= 0.5 * theta ** 2 * np.abs(want4).max()


def _one_step_error(scheme, c, theta, n):
    J = np.arange(n)
    g = np.cos(theta * J)
    exact = np.cos(theta * (J - c))  # translation by c nodes
    return np.abs(g + O.fd_convection_update(g, c, 0, scheme) - exact).max()


def test_lw_error_is_the_dispersion_term_and_r3_removes_it():
    n, c = 8192, 0.3
    ths, e_lw, e_1 = [], [], []
    for m in (16, 32, 64, 128):
        th = 2.0 * np.pi * m / n
        ths.append(th)
        e_lw.append(_one_step_error(O.LAX_WENDROFF, c, th, n))
        e_1.append(_one_step_error(O.MLW1, c, th, n))
    lt = np.log(ths)
    slope_lw = np.polyfit(lt, np.log(e_lw), 1)[0]
    slope_1 = np.polyfit(lt, np.log(e_1), 1)[0]
    assert abs(slope_lw - 3.0) < 0.1, slope_lw
    assert abs(slope_1 - 4.0) < 0.1, slope_1
    # the LW error's size is the dispersion term: c (1 - c^2) theta^3 / 6
    assert e_lw[0] == pytest.approx(c * (1 - c * c) * ths[0] ** 3 / 6.0, rel=0.02)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_small_cfl_tends_to_central_difference(scheme):
    # LW -> minus the second-order central difference (g[J+1] - g[J-1]) / 2; with R3 (of
    # order c) the limit is minus the fourth-order central difference
    # (8 (g[J+1] - g[J-1]) - (g[J+2] - g[J-2])) / 12
    g = _profile(32, seed=9)
    gp1, gm1, gp2, gm2 = (np.roll(g, s) for s in (-1, 1, -2, 2))
    cd = -(8.0 * (gp1 - gm1) - (gp2 - gm2)) / 12.0 if scheme >= O.MLW1 else -0.5 * (gp1 - gm1)
    c = 1e-7
    assert np.allclose(O.fd_convection_update(g, c, 0, scheme) / c, cd, atol=1e-6)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_step_convection_acts_per_axis(scheme):
    # population q = 3 (speed group 1, direction i = 3) moves along +y only
    ny, nx = 8, 16
    rng = np.random.default_rng(2)
    f = 1.0 + 0.01 * rng.standard_normal((O.Q, ny, nx))
    p = O.Params(conv=scheme, m=O.CENTRAL_DIFFERENCE)
    v = O.velocities()
    q = 3
    assert abs(v[q, 0]) < 1e-12 and v[q, 1] > 0
    D = O.Deriv(ny, nx, p)
    C = O.convection(f, v, D, p)
    du_y = O.fd_convection_update(f[q], v[q, 1] * p.dt / p.dy, 0, scheme)
    assert np.allclose(-p.dt * C[q], du_y, rtol=0, atol=1e-15)
    # population q = 1 moves along +x only
    du_x = O.fd_convection_update(f[1], v[1, 0] * p.dt / p.dx, 1, scheme)
    assert np.allclose(-p.dt * C[1], du_x, rtol=0, atol=1e-15)
    assert np.all(C[0] == 0.0)


def test_unknown_scheme_rejected():
    with pytest.raises(ValueError):
        O.fd_convection_update(np.zeros(8), 0.1, 0, 4)


# ---------------------------------------------------------------------------
# Flux limiter (Sec. 3.1, MCD limiter along characteristic lines)
# ---------------------------------------------------------------------------

AXES = [(1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]


def _field(ny=12, nx=16, seed=7):
    return np.random.default_rng(seed).standard_normal((ny, nx))


@pytest.mark.parametrize("e", AXES)
def test_fl_unit_cfl_is_an_exact_shift(e):
    # c = 1: F_{J+1/2} = g_J whatever psi, so g moves one node along e
    g = _field()
    out = g + O.fl_convection_update(g, 1.0, e)
    assert np.allclose(out, O._along(g, e, -1), rtol=0, atol=1e-13)


@pytest.mark.parametrize("e", [(1, 0), (0, 1), (-1, 0), (0, -1)])
def test_fl_limiter_one_is_lax_wendroff_and_zero_is_upwind(e):
    # the paper: psi = 1 gives the LW scheme, psi = 0 the first-order upwind scheme
    g = _field()
    c = 0.37
    axis = 1 if e[0] else 0
    cs = c * (e[0] or e[1])     # signed CFL number along the axis
    lw = O.fl_convection_update(g, c, e, limiter=lambda t: np.ones_like(t))
    assert np.allclose(lw, O.fd_convection_update(g, cs, axis, O.LAX_WENDROFF), rtol=0, atol=1e-13)
    up = O.fl_convection_update(g, c, e, limiter=lambda t: np.zeros_like(t))
    assert np.allclose(up, -c * (g - O._along(g, e, -1)), rtol=0, atol=1e-13)


def test_mcd_limiter_values():
    th = np.array([-1.0, 0.0, 0.1, 1.0 / 3.0, 0.5, 1.0, 3.0, 5.0])
    want = np.array([0.0, 0.0, 0.2, 2.0 / 3.0, 0.75, 1.0, 2.0, 2.0])
    assert np.allclose(O.mcd_limiter(th), want, rtol=0, atol=1e-15)


@pytest.mark.parametrize("e", [(1, 0), (1, 1)])
def test_fl_is_total_variation_diminishing(e):
    # a square pulse advected 200 steps at c = 0.6: no new extrema, variation does not grow
    ny, nx = 8, 64
    g = np.zeros((ny, nx))
    g[:, 20:30] = 1.0
    g[2:5, :] += 0.5 * (e[1] != 0)
    tv0 = np.abs(np.diff(g, axis=1)).sum()
    lo, hi = g.min(), g.max()
    for _ in range(200):
        g = g + O.fl_convection_update(g, 0.6, e)
        assert g.min() >= lo - 1e-12 and g.max() <= hi + 1e-12
    if e == (1, 0):
        assert np.abs(np.diff(g, axis=1)).sum() <= tv0 + 1e-12


def test_fl_conserves_the_sum_and_is_second_order_on_smooth_data():
    for e in AXES:
        g = _field(seed=11)
        assert abs(O.fl_convection_update(g, 0.4, e).sum()) < 1e-12
    # one step of a smooth wave along x: error against exact translation falls ~ 4x per halving
    errs = []
    for n in (64, 128, 256):
        x = np.arange(n) / n
        g = np.tile(np.sin(2 * np.pi * x) + 2.0, (4, 1))
        c = 0.5
        steps = n // 8                      # the same physical time
        for _ in range(steps):
            g = g + O.fl_convection_update(g, c, (1, 0))
        exact = np.sin(2 * np.pi * (x - c * steps / n)) + 2.0
        errs.append(np.abs(g[0] - exact).mean())
    order = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
    assert min(order) > 1.5, order


def test_fl_step_uses_each_population_s_line():
    ny, nx = 8, 16
    rng = np.random.default_rng(3)
    f = 1.0 + 0.01 * rng.standard_normal((O.Q, ny, nx))
    p = O.Params(conv=O.FLUX_LIMITER, m=O.CENTRAL_DIFFERENCE)
    v = O.velocities()
    C = O.convection(f, v, O.Deriv(ny, nx, p), p)
    for q in (1, 2, 4, 10):
        e, A = O.characteristic(v[q])
        c = math.hypot(*v[q]) * p.dt / (A * p.dx)
        assert np.allclose(-p.dt * C[q], O.fl_convection_update(f[q], c, e), rtol=0, atol=1e-15)
    assert O.characteristic(v[2]) == ((1, 1), math.sqrt(2.0))
