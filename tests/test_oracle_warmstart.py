"""Pins of the warm-start transform and of the energy match in the FP64 oracle (no GPU).

The transform (clip, binomial filter, interface mass shift, uniform temperature) and the
energy match are not in the paper: they prepare the start of a run from the warm-start
network's prediction.  They are pinned to closed forms (the filter's transfer function,
central differences of a sinusoid, the energy of a uniform state), to invariants (exact
mass and energy) and to an independent route (root finding instead of the linearity
argument)."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import cnn_oracle as C
from oracle import fftlb_oracle as O


def test_binomial_filter_transfer_function():
    # (1 2 1)/4 multiplies the mode cos(2 pi p x / N) by (1 + cos(2 pi p / N)) / 2 = cos^2(pi p / N)
    ny, nx = 12, 16
    x = np.arange(nx)[None, :]
    y = np.arange(ny)[:, None]
    for p, q in [(0, 0), (1, 0), (3, 2), (8, 0), (0, 6), (5, 5)]:
        g = np.cos(2 * np.pi * p * x / nx + 0.3) * np.cos(2 * np.pi * q * y / ny - 0.7)
        want = np.cos(np.pi * p / nx) ** 2 * np.cos(np.pi * q / ny) ** 2 * g
        assert np.abs(C.binomial_filter(g) - want).max() < 1e-14


def test_binomial_filter_conserves_the_sum_and_kills_nyquist():
    rng = np.random.default_rng(0)
    g = rng.uniform(0.2, 1.5, (16, 24))
    assert C.binomial_filter(g).sum() == pytest.approx(g.sum(), rel=1e-14)
    checker = (-1.0) ** np.arange(24)[None, :] * np.ones((16, 1))
    assert np.abs(C.binomial_filter(checker)).max() < 1e-15
    assert np.array_equal(C.binomial_filter(np.full((8, 8), 0.7)), np.full((8, 8), 0.7))


def test_interface_weight_of_sinusoids():
    n = 32
    x = np.arange(n)
    rho = np.sin(2 * np.pi * x / n)[None, :].repeat(8, 0)
    want = np.abs(np.sin(2 * np.pi / n) * np.cos(2 * np.pi * x / n))[None, :]
    assert np.abs(C.interface_weight(rho) - want).max() < 1e-14
    assert np.abs(C.interface_weight(rho.T) - want.T).max() < 1e-14


def _droplet(n, radius, rho_v, rho_l, width=2.0):
    y, x = np.mgrid[0:n, 0:n]
    r = np.hypot(x - n / 2, y - n / 2)
    return 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh((r - radius) / width)


RHO_C, T_C = 5.0 / 6.0, 8 * 2.0 / (27 * 0.4)


def test_transform_restores_mass_at_the_interfaces():
    n = 64
    rho0 = _droplet(n, 14, 0.27, 1.50, 4.0)          # the run's initial field
    pred_rho = _droplet(n, 13, 0.25, 1.55, 1.5)      # a sharper, smaller, denser prediction
    pred = np.stack([pred_rho / RHO_C, np.full((n, n), 0.85)])
    rho, T = C.warm_start_transform(pred, rho0, RHO_C, T_C, 0.95 / 0.4)
    assert rho.sum() == pytest.approx(rho0.sum(), rel=1e-13)
    assert np.all(T == T[0, 0]) and T[0, 0] == pytest.approx(0.85 * T_C, rel=1e-14)
    # the deficit went to the interfaces: the bulks keep the filtered prediction
    filt = C.binomial_filter(pred_rho)
    core, far = (n // 2, n // 2), (2, 2)
    assert abs(rho[core] - filt[core]) < 2e-3 * filt[core] and abs(rho[far] - filt[far]) < 2e-3 * filt[far]
    w = C.interface_weight(filt)
    ring = w > 0.1 * w.max()
    deficit = rho0.sum() - filt.sum()
    assert deficit > 0.05 * rho0.sum()
    assert (rho[ring] - filt[ring]).sum() > 0.9 * deficit


def test_transform_of_a_field_without_interfaces_is_uniform():
    n = 16
    rho0 = np.full((n, n), 0.9)
    pred = np.stack([np.full((n, n), 1.3 / RHO_C), np.full((n, n), 0.9)])
    rho, T = C.warm_start_transform(pred, rho0, RHO_C, T_C, 0.95 / 0.4)
    assert np.abs(rho - 0.9).max() < 1e-15
    assert np.abs(T - 0.9 * T_C).max() < 1e-15


def test_transform_clips_to_the_physical_range():
    n = 32
    rng = np.random.default_rng(3)
    rho0 = _droplet(n, 8, 0.3, 1.4)
    noisy = rho0 * rng.uniform(0.9, 1.1, (n, n))
    noisy[3, 4], noisy[20, 9], noisy[11, 30] = 7.0, -2.0, 3.0      # outliers beyond both bounds
    pred = np.stack([noisy / RHO_C, rng.uniform(-0.5, 0.0, (n, n))])
    rho_max = 0.95 / 0.4
    rho, T = C.warm_start_transform(pred, rho0, RHO_C, T_C, rho_max)
    assert rho.sum() == pytest.approx(rho0.sum(), rel=1e-13)
    lo, hi = C.RHO_MIN_FRACTION * RHO_C, rho_max
    assert rho.min() > 0.99 * lo and rho.max() < 1.01 * hi           # up to the final mass rescale
    assert np.all(T == C.T_MIN_FRACTION * T_C)       # the predicted mean temperature is below the floor


P = O.Params(dx=1 / 256, dy=1 / 256, dt=1e-5, tau=1e-2, K=1e-5, H=0.0, zeta=0.0, q=-0.004, a=2.0, b=0.4, m=4)


def test_energy_match_of_a_uniform_state_closed_form():
    n = 16
    rho, ux, uy = np.full((n, n), 0.8), np.full((n, n), 0.05), np.full((n, n), -0.02)
    T = np.full((n, n), 1.1)
    E0 = 0.123
    cells = n * n * P.dx * P.dy
    # E = cells (rho T - a rho^2 + rho |u|^2 / 2), solved for T
    want = E0 / (cells * 0.8) + P.a * 0.8 - 0.5 * (0.05 ** 2 + 0.02 ** 2)
    assert np.abs(O.match_energy(rho, ux, uy, T, E0, P) - want).max() < 1e-12


def test_energy_match_agrees_with_root_finding_and_the_distribution():
    n = 48
    rho = _droplet(n, 11, 0.27, 1.5, 1.5)
    z = np.zeros_like(rho)
    T = np.full_like(rho, 1.25)
    E0 = O.fields_energy(rho, z, z, T, P) + 0.01
    Tm = O.match_energy(rho, z, z, T, E0, P)
    assert np.all(Tm == Tm[0, 0])
    root = brentq(lambda t: O.fields_energy(rho, z, z, np.full_like(rho, t), P) - E0, 0.5, 2.0, xtol=1e-15)
    assert Tm[0, 0] == pytest.approx(root, rel=1e-12)
    # the state f^eq(rho, 0, Tm) has that energy by the moment route too
    assert O.globals_of(O.feq(rho, z, z, Tm), P)["energy"] == pytest.approx(E0, rel=1e-11)
