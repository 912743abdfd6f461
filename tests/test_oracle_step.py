"""Pins of the oracle's time step (Sec. 3, Eq. (24) form with the WFFT of Sec. 3.6).

  * A uniform state, at rest or moving, is a fixed point (all derivatives vanish).
  * Mass and momentum are conserved (collision and force conserve them locally or
    globally; every windowed derivative has zero mean).
  * Free streaming (no collision, ideal gas): a Fourier mode of f_q is multiplied by
    (1 - i dt v_q.k_m) per step, exactly.
"""
import math

import numpy as np
import pytest

from oracle import fftlb_oracle as O
from paper_1011_3582_amd import workloads as W


def _params(**kw):
    p = W.model_params()
    p.update(kw)
    return O.Params(**p)


@pytest.mark.parametrize("u", [(0.0, 0.0), (0.12, -0.05)])
def test_uniform_state_is_fixed_point(u):
    p = _params()
    fld = W.uniform(16, 16, rho=0.9, ux=u[0], uy=u[1], T=1.2)
    f0 = O.init_distribution(*fld.as_f64())
    f = O.run(f0, p, 20)
    np.testing.assert_allclose(f, f0, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("case", ["slab", "smooth"])
def test_mass_and_momentum_conserved(case):
    p = _params()
    if case == "slab":
        fld = W.slab(32, 16, t_ratio=0.9, noise=1e-3, seed=3)
    else:
        fld = W.smooth_random(32, 32, seed=5, T0=1.2)
    f0 = O.init_distribution(*fld.as_f64())
    g0 = O.globals_of(f0, p)
    f = O.run(f0, p, 30)
    g1 = O.globals_of(f, p)
    assert g1["mass"] == pytest.approx(g0["mass"], rel=1e-13)
    scale = g0["mass"] * math.sqrt(1.2)
    assert abs(g1["px"] - g0["px"]) < 1e-13 * scale
    assert abs(g1["py"] - g0["py"]) < 1e-13 * scale


def test_free_streaming_mode_amplification():
    """tau = inf, a = b = K = q = 0: f_q^{n+1} = f_q^n - dt v_q . grad_m f_q^n with I = 0."""
    ny, nx = 8, 16
    p = O.Params(dx=0.05, dy=0.04, dt=2e-3, tau=math.inf, K=0.0, H=0.0, zeta=0.0, q=0.0, a=0.0, b=0.0, m=3)
    x = np.arange(nx)[None, :] * p.dx
    y = np.arange(ny)[:, None] * p.dy
    kx_i, ky_i = 3, -2
    kx, ky = 2 * np.pi * kx_i / (nx * p.dx), 2 * np.pi * ky_i / (ny * p.dy)
    rng = np.random.default_rng(9)
    amp = rng.normal(size=33) + 1j * rng.normal(size=33)
    base = 1.0 + rng.uniform(0.5, 1.0, size=33)
    phase = np.exp(1j * (kx * x + ky * y))
    f0 = np.stack([base[q] + 0.01 * (amp[q] * phase).real for q in range(33)])
    n = 7
    f = O.run(f0, p, n)
    v = O.velocities()
    s = lambda k, d: 2 / d * sum(c * math.sin(k * d / 2) ** (2 * j + 1)
                                 for j, c in enumerate([1, 1 / 6, 3 / 40, 5 / 112][:p.m]))
    for q in range(33):
        g = (1 - 1j * p.dt * (v[q, 0] * s(kx, p.dx) + v[q, 1] * s(ky, p.dy))) ** n
        ref = base[q] + 0.01 * (amp[q] * g * phase).real
        np.testing.assert_allclose(f[q], ref, rtol=0, atol=1e-13)


def test_step_reduces_to_bgk_without_gradients_of_force_inputs():
    """On a uniform density and temperature with a sheared velocity the force's pressure
    parts vanish; the step must still conserve mass exactly and move momentum only by
    divergences (zero mean)."""
    p = _params()
    ny, nx = 16, 16
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    ux = 0.05 * np.sin(2 * np.pi * y / ny)
    f0 = O.feq(np.ones((ny, nx)), ux, np.zeros((ny, nx)), np.full((ny, nx), 1.1))
    parts = O.step_parts(f0, p)
    assert abs(parts.I.sum()) < 1e-12
    assert abs(parts.conv.sum()) < 1e-9


def test_momentum_residual_equals_convection_sum():
    """dt max|D.(rho u)| of a state equals dt max|sum_q C_q| of its convection terms: the
    windowed derivative is linear and sum_q v_q f_q = rho u; two independent routes."""
    p = _params()
    rng = np.random.default_rng(11)
    ny, nx = 24, 32
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * 3 * x / nx)
    f = O.feq(rho, 0.05 * np.cos(2 * np.pi * x / nx), np.zeros((ny, nx)), np.full((ny, nx), 1.2))
    f = f * (1.0 + 0.01 * rng.uniform(-1, 1, f.shape))      # off equilibrium, all modes present
    parts = O.step_parts(f, p)
    r_conv = O.residual(parts.conv, p)
    r_mom = O.momentum_residual(f, p)
    assert r_conv > 1e-6
    assert r_mom == pytest.approx(r_conv, rel=1e-12)


def test_momentum_residual_of_a_single_mode():
    """A momentum field rho u_x = A sin(k x) with rho = 1 has D.(rho u) = A k_m cos(k x)."""
    p = _params()
    ny, nx, n = 8, 64, 5
    x = np.arange(nx)[None, :] * np.ones((ny, 1))
    k = 2 * np.pi * n / (nx * p.dx)
    A = 0.01
    f = O.feq(np.ones((ny, nx)), A * np.sin(k * x * p.dx), np.zeros((ny, nx)), np.full((ny, nx), 1.0))
    km = O.kappa(nx, p.dx, p.m)[n]
    assert O.momentum_residual(f, p) == pytest.approx(p.dt * A * km, rel=1e-9)
