"""Pins of the oracle's NPS stencils (Sec. 3.1: nine-point first derivative with B = 1/12 and
Laplacian with F = 1/6) against facts fixed outside their code:

  * the truncation errors the paper states for them,
      D_x = d_x + (1/6) dx^2 d_x^3 + 2 B dx^2 d_x d_y^2 + ...,
      Lap = lap + (dx^2/12)(d_x^4 + d_y^4) + F dx^2 d_x^2 d_y^2 + ...,
    checked on a smooth periodic field to leading order;
  * the isotropy these weights were chosen for: on two plane waves of equal |k| in different
    directions, (5, 0) and (3, 4), the Laplacian and the gradient magnitude agree to leading
    order (the central difference's Laplacian does not);
  * the stencils conserve the sum over the periodic grid.
"""
import numpy as np
import pytest

from oracle import fftlb_oracle as O


def _grid(n):
    d = 2.0 * np.pi / n
    x = np.arange(n) * d
    X, Y = np.meshgrid(x, x)   # [y, x]
    return d, X, Y


def _deriv(n, d, m=O.NPS):
    return O.Deriv(n, n, O.Params(dx=d, dy=d, m=m))


def test_first_derivative_truncation_error():
    n = 256
    d, X, Y = _grid(n)
    g = np.sin(3 * X) * np.cos(5 * Y)
    D = _deriv(n, d)
    err = D.x(g) - 3 * np.cos(3 * X) * np.cos(5 * Y)
    # (1/6) d^2 g_xxx + 2 B d^2 g_xyy, g_xxx = -27 cos3x cos5y, g_xyy = -75 cos3x cos5y
    lead = d * d * (-27.0 / 6.0 + 2.0 * O.NPS_B * -75.0) * np.cos(3 * X) * np.cos(5 * Y)
    assert np.abs(err - lead).max() < 0.02 * np.abs(lead).max()
    err_y = D.y(g) + 5 * np.sin(3 * X) * np.sin(5 * Y)
    # (1/6) d^2 g_yyy + 2 B d^2 g_yxx, g_yyy = 125 sin3x sin5y, g_yxx = 45 sin3x sin5y
    lead_y = d * d * (125.0 / 6.0 + 2.0 * O.NPS_B * 45.0) * np.sin(3 * X) * np.sin(5 * Y)
    assert np.abs(err_y - lead_y).max() < 0.02 * np.abs(lead_y).max()


def test_laplacian_truncation_error():
    n = 256
    d, X, Y = _grid(n)
    g = np.sin(3 * X) * np.cos(5 * Y)
    D = _deriv(n, d)
    err = D.laplacian(g) - (-34.0 * g)
    lead = d * d * ((81.0 + 625.0) / 12.0 + O.NPS_F * 225.0) * g
    assert np.abs(err - lead).max() < 0.02 * np.abs(lead).max()


@pytest.mark.parametrize("m,isotropic", [(O.NPS, True), (O.CENTRAL_DIFFERENCE, False)])
def test_laplacian_isotropy(m, isotropic):
    n = 128
    d, X, Y = _grid(n)
    D = _deriv(n, d, m)
    errs = []
    for kx, ky in ((5, 0), (3, 4)):
        g = np.cos(kx * X + ky * Y)
        lap = D.laplacian(g)
        errs.append(float(np.abs(lap + 25.0 * g).max()))
    spread = abs(errs[0] - errs[1]) / max(errs)
    if isotropic:
        assert spread < 0.05, errs   # next order: relative O(k^2 d^2)
    else:
        assert spread > 0.3, errs


def test_gradient_isotropy():
    n = 128
    d, X, Y = _grid(n)
    D = _deriv(n, d)
    ratios = []
    for kx, ky in ((5, 0), (3, 4)):
        g = np.sin(kx * X + ky * Y)
        gx, gy = D.x(g), D.y(g)
        ratios.append(float(np.sqrt(gx ** 2 + gy ** 2).max()) / 5.0)
    # both ratios are 1 - (d^2/6) |k|^2 to leading order
    lead = 25.0 * d * d / 6.0
    assert ratios[0] == pytest.approx(1.0 - lead, rel=0.1 * lead)
    assert abs(ratios[0] - ratios[1]) < 0.05 * lead


def test_stencils_conserve_the_sum():
    rng = np.random.default_rng(4)
    g = rng.standard_normal((12, 20))
    D = O.Deriv(12, 20, O.Params(dx=0.1, dy=0.1, m=O.NPS))
    for out in (D.x(g), D.y(g), D.laplacian(g)):
        assert abs(out.sum()) < 1e-11


def test_nps_needs_a_square_lattice():
    with pytest.raises(ValueError):
        O.Deriv(8, 8, O.Params(dx=0.1, dy=0.2, m=O.NPS))
