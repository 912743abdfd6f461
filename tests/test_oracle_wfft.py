"""Pins of the oracle's windowed-FFT derivative operator (Sec. 3.6 and Appendix A).

The operator is checked against a brute-force evaluation of the paper's transform
pair, exact derivatives of sinusoids, the half-step central difference that k_1
reduces to, the arcsin series, and the orders and leading error constants of
the four windows.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import fftlb_oracle as O

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _params(m, dx=1.0 / 256, dy=None):
    return O.Params(dx=dx, dy=dx if dy is None else dy, m=m)


def _brute_deriv(g, axis, m, dx, dy):
    """Eq. (40) forward transform (with the dx dy factor), multiply by i k_m (Eq. (42) with the
    window of Eqs. (44)-(47)), Eq. (41) inverse sum over n = -N/2..N/2-1 with 1/(Lx Ly),
    all by explicit O(N^4) sums."""
    ny, nx = g.shape
    Lx, Ly = nx * dx, ny * dy
    xs = np.arange(nx) * dx
    ys = np.arange(ny) * dy
    nxs = np.arange(-nx // 2, nx // 2)
    nys = np.arange(-ny // 2, ny // 2)
    kxs = 2 * np.pi * nxs / Lx
    kys = 2 * np.pi * nys / Ly

    def window(k, n, N, d):
        if m == 0:
            kap = k.copy()
        else:
            s = np.sin(k * d / 2)
            kap = sum(c * s ** (2 * j + 1) for j, c in enumerate(GOLDEN["arcsin_coefficients"]["value"][:m])) * 2 / d
        kap[n == -N // 2] = 0.0      # Nyquist reading
        return kap

    out = np.zeros((ny, nx))
    for iy, ky in enumerate(kys):
        for ix, kx in enumerate(kxs):
            ft = dx * dy * np.sum(g * np.exp(-1j * (kx * xs[None, :] + ky * ys[:, None])))
            mult = 1j * (window(kxs, nxs, nx, dx)[ix] if axis == "x" else window(kys, nys, ny, dy)[iy])
            out += ((mult * ft) * np.exp(1j * (kx * xs[None, :] + ky * ys[:, None]))).real / (Lx * Ly)
    return out


@pytest.mark.parametrize("ny,nx", [(4, 4), (6, 8), (8, 6), (12, 12), (16, 8)])
@pytest.mark.parametrize("m", [0, 1, 4])
def test_derivative_matches_brute_force_transform_pair(ny, nx, m):
    rng = np.random.default_rng(ny * 100 + nx + m)
    g = rng.normal(size=(ny, nx))
    p = _params(m, dx=0.1, dy=0.07)
    D = O.Deriv(ny, nx, p)
    for axis, op in (("x", D.x), ("y", D.y)):
        ref = _brute_deriv(g, axis, m, p.dx, p.dy)
        np.testing.assert_allclose(op(g), ref, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("m", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("p_mode", [1, 5, 31])
def test_derivative_of_sinusoid(m, p_mode):
    """D sin(2 pi p x/L + phi) = k_m(2 pi p/L) cos(...) exactly; m = 0 is the exact derivative."""
    n, dx = 64, 1.0 / 256
    L = n * dx
    x = np.arange(n) * dx
    k = 2 * np.pi * p_mode / L
    g = np.sin(k * x + 0.3)[None, :].repeat(8, 0)
    D = O.Deriv(8, n, _params(m, dx=dx))
    s = math.sin(k * dx / 2)
    coeffs = [math.comb(2 * j, j) / (4 ** j * (2 * j + 1)) for j in range(4)]   # arcsin series
    kap = k if m == 0 else 2 / dx * sum(coeffs[j] * s ** (2 * j + 1) for j in range(m))
    ref = np.broadcast_to(kap * np.cos(k * x + 0.3)[None, :], g.shape)
    np.testing.assert_allclose(D.x(g), ref, atol=1e-12 * k)
    # along y the same field is constant
    np.testing.assert_allclose(D.y(g), 0 * g, atol=1e-12 * k)


def test_nyquist_mode_is_annihilated():
    n = 32
    g = np.cos(np.pi * np.arange(n))[None, :].repeat(4, 0)    # the Nyquist mode
    for m in range(5):
        D = O.Deriv(4, n, _params(m))
        assert np.abs(D.x(g)).max() < 1e-12


def test_window_coefficients_are_arcsin_series():
    """Eqs. (43)-(47): the coefficients are those of arcsin s = sum (2j)!/(4^j (j!)^2 (2j+1)) s^(2j+1)."""
    for j, c in enumerate(O.ARCSIN_COEFFS):
        assert c == pytest.approx(math.comb(2 * j, j) / (4 ** j * (2 * j + 1)), rel=1e-15)
        assert c == pytest.approx(GOLDEN["arcsin_coefficients"]["value"][j], rel=1e-15)
    # with many terms the series returns k itself (|k dx/2| < pi/2)
    n, dx = 64, 0.01
    k = O.wavenumbers(n, dx)
    s = np.sin(k * dx / 2)
    full = 2 / dx * sum(math.comb(2 * j, j) / (4 ** j * (2 * j + 1)) * s ** (2 * j + 1) for j in range(400))
    inner = np.abs(k * dx / 2) < 1.2
    np.testing.assert_allclose(full[inner], k[inner], rtol=1e-12)


def test_k1_smoothing_factor_is_sinc():
    """Eq. (48): sigma_1 = k_1/k = sin(n pi/N)/(n pi/N)."""
    n, dx = 128, 1.0 / 256
    k = O.wavenumbers(n, dx)
    kap = O.kappa(n, dx, 1)
    nn = np.fft.fftfreq(n) * n
    sel = (nn != 0) & (nn != -n // 2)
    np.testing.assert_allclose(kap[sel] / k[sel], np.sin(nn[sel] * np.pi / n) / (nn[sel] * np.pi / n), rtol=1e-14)


def test_k1_is_half_step_central_difference():
    """Appendix A: IFT[i k_1 FT f] = (f(x + dx/2) - f(x - dx/2))/dx on band-limited data."""
    n, dx = 48, 0.05
    L = n * dx
    x = np.arange(n) * dx
    rng = np.random.default_rng(7)
    modes = rng.integers(1, n // 2, size=6)
    amps = rng.normal(size=6)
    phs = rng.uniform(0, 2 * np.pi, size=6)
    f = lambda xx: sum(a * np.sin(2 * np.pi * p * xx / L + ph) for a, p, ph in zip(amps, modes, phs))
    D = O.Deriv(2, n, _params(1, dx=dx))
    got = D.x(f(x)[None, :].repeat(2, 0))[0]
    ref = (f(x + dx / 2) - f(x - dx / 2)) / dx
    np.testing.assert_allclose(got, ref, atol=1e-12 * np.abs(ref).max())


def _sin_error(n, m):
    L = 2 * np.pi
    dx = L / n
    x = np.arange(n) * dx
    D = O.Deriv(2, n, _params(m, dx=dx))
    return np.abs(D.x(np.sin(x)[None, :].repeat(2, 0))[0] - np.cos(x)).max()


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_orders_of_accuracy(m):
    """Appendix A: k_1..k_4 give orders 2, 4, 6, 8.  The leading error of k_m on sin(x) is
    e_m dx^(2m) with e_m = c_m / 4^m (c_m the (m+1)-th arcsin coefficient): 1/24, 3/640,
    5/7168, 35/294912.  (The Appendix prints 1/1920, 1/322560, 1/92897280 for m = 2, 3, 4;
    those are the higher Taylor terms of the k_1 half-step difference, not the leading
    errors of k_2..k_4.)"""
    order = GOLDEN["accuracy_orders"]["value"][str(m)]
    assert order == 2 * m
    c_next = math.comb(2 * m, m) / (4 ** m * (2 * m + 1))
    e_m = c_next / 4 ** m
    assert e_m == pytest.approx([1 / 24, 3 / 640, 5 / 7168, 35 / 294912][m - 1], rel=1e-14)
    n = 64 if m < 4 else 16
    err1, err2 = _sin_error(n, m), _sin_error(2 * n, m)
    if m < 4:
        assert err1 / err2 == pytest.approx(2 ** order, rel=0.02)
    dx = 2 * np.pi / n
    assert err1 == pytest.approx(e_m * dx ** order, rel=0.05)


def test_k4_reaches_round_off_on_sin():
    """Sec. 3.6 (Fig. 5 discussion): with k_4 the error of d/dx sin(x) at N = 128 is round-off."""
    assert _sin_error(128, 4) < 1e-13
    assert _sin_error(128, 1) > 1e-5


def test_central_difference_of_a_sinusoid_and_its_order():
    """The central-difference operator (m = 5, Sec. 3.1): on sin(p x) it gives
    sin(p dx)/dx cos(p x) exactly, the symbol kappa returns; its error is -dx^2/6 f''' to
    leading order (second order: halving dx divides it by 4)."""
    from oracle import fftlb_oracle as O
    errs = []
    for n in (64, 128):
        L = 2 * np.pi
        dx = L / n
        p = O.Params(dx=dx, dy=dx, dt=1e-5, tau=1e-2, K=0.0, H=0.0, zeta=0.0, q=0.0, a=0.0, b=0.0,
                     m=O.CENTRAL_DIFFERENCE)
        D = O.Deriv(8, n, p)
        x = np.arange(n) * dx
        g = np.sin(3 * x + 0.2)[None, :].repeat(8, 0)
        got = D.x(g)
        assert np.abs(got - np.sin(3 * dx) / dx * np.cos(3 * x + 0.2)).max() < 1e-12
        assert O.kappa(n, dx, O.CENTRAL_DIFFERENCE)[3] == pytest.approx(np.sin(3 * dx) / dx, rel=1e-14)
        errs.append(np.abs(got - 3 * np.cos(3 * x + 0.2)).max())
        # leading error -dx^2/6 f''' = -dx^2/6 * (-27 cos) at this resolution
        assert errs[-1] == pytest.approx(27 * dx * dx / 6 * 1.0, rel=0.02)
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.01)


def test_central_difference_convection_equals_its_symbol():
    """The stencil convection of the oracle (real space) equals the spectral product with
    the central-difference symbol i (v_x sin(k_x dx)/dx + v_y sin(k_y dy)/dy): the two routes
    agree to round-off (the HIP path uses the spectral one)."""
    from oracle import fftlb_oracle as O
    rng = np.random.default_rng(5)
    ny, nx = 16, 24
    p = O.Params(dx=1 / 256, dy=1 / 200, dt=1e-5, tau=1e-2, K=1e-5, H=0.0, zeta=0.0, q=-0.004, a=2.0, b=0.4,
                 m=O.CENTRAL_DIFFERENCE)
    f = rng.uniform(0.1, 1.0, (33, ny, nx))
    D = O.Deriv(ny, nx, p)
    v = O.velocities()
    got = O.convection(f, v, D)
    kx = O.kappa(nx, p.dx, p.m)[None, :]
    ky = O.kappa(ny, p.dy, p.m)[:, None]
    for q in range(1, 33):
        ref = np.fft.ifft2(1j * (v[q, 0] * kx + v[q, 1] * ky) * np.fft.fft2(f[q])).real
        assert np.abs(got[q] - ref).max() < 1e-12 * np.abs(ref).max() + 1e-12


@pytest.mark.parametrize("m", [0, 1, 4, O.CENTRAL_DIFFERENCE])
def test_convection_splits_by_axis_into_one_dimensional_derivatives(m):
    """The convection term of Sec. 3.6 (one 2D transform pair with the multiplier
    i (v_x k_m(kx) + v_y k_m(ky))) equals v_x times the 1D windowed derivative along each row plus
    v_y times the 1D windowed derivative along each column, each formed with 1D transforms: the
    multiplier is a sum of one-axis multipliers.  The 1D derivatives also pass two real rows (or
    columns) at once as one complex sequence a + i b: the multiplier is odd and zero at the
    Nyquist bin, so the result is D a + i D b.  (The HIP path forms the parts this way.)"""
    ny, nx = 24, 40
    p = O.Params(dx=1.0 / 40, dy=1.0 / 36, m=m)
    rng = np.random.default_rng(17 + m)
    f = rng.uniform(0.0, 1.0, (3, ny, nx))
    v = np.array([[0.0, 0.0], [1.9 * 0.7071, 1.9 * 0.7071], [-2.9, 0.0]])
    D = O.Deriv(ny, nx, p)
    conv = O.convection(f, v, D)
    kx = O.kappa(nx, p.dx, m) if m != O.CENTRAL_DIFFERENCE else np.sin(O.wavenumbers(nx, p.dx) * p.dx) / p.dx
    ky = O.kappa(ny, p.dy, m) if m != O.CENTRAL_DIFFERENCE else np.sin(O.wavenumbers(ny, p.dy) * p.dy) / p.dy
    kx[nx // 2] = 0.0
    ky[ny // 2] = 0.0

    def d1(z, k, axis):
        Z = np.fft.fft(z, axis=axis)
        shape = [1, 1]
        shape[axis] = -1
        return np.fft.ifft(1j * k.reshape(shape) * Z, axis=axis)

    for q in (1, 2):
        dx_rows = d1(f[q], kx, 1).real
        dy_cols = d1(f[q], ky, 0).real
        np.testing.assert_allclose(conv[q], v[q, 0] * dx_rows + v[q, 1] * dy_cols, rtol=0, atol=1e-11 * np.abs(conv[q]).max())
        # two real rows as one complex row, two real columns as one complex column
        pr = d1(f[q] + 1j * f[q + 1 if q < 2 else 1], kx, 1)
        np.testing.assert_allclose(pr.real, dx_rows, rtol=0, atol=1e-11 * np.abs(dx_rows).max())
        np.testing.assert_allclose(pr.imag, d1(f[q + 1 if q < 2 else 1], kx, 1).real, rtol=0,
                                   atol=1e-11 * np.abs(dx_rows).max())
        pc = d1(f[q][:, 0::2] + 1j * f[q][:, 1::2], ky, 0)
        np.testing.assert_allclose(pc.real, dy_cols[:, 0::2], rtol=0, atol=1e-11 * np.abs(dy_cols).max())
        np.testing.assert_allclose(pc.imag, dy_cols[:, 1::2], rtol=0, atol=1e-11 * np.abs(dy_cols).max())
    # the rest population has no convection term
    assert np.all(conv[0] == 0.0)
