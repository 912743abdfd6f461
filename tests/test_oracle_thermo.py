"""Pins of the van der Waals thermodynamics used by the oracle's tests and by the
workload generators (Sec. 4.1 coexistence curve, Sec. 4.2 Laplace law)."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import thermo
from paper_1011_3582_amd import workloads as W

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_coexistence_matches_printed_values():
    g = GOLDEN["coexistence_T0.99"]
    rv, rl = thermo.maxwell(g["T"], g["a"], g["b"])
    tol = 0.5 * 10 ** -g["printed_digits"]
    assert abs(rv - g["rho_v"]) <= tol and abs(rl - g["rho_l"]) <= tol
    g = GOLDEN["droplet_T0.95"]
    rv, rl = thermo.maxwell(g["T"], g["a"], g["b"])
    tol = 0.5 * 10 ** -g["printed_digits"]
    assert abs(rv - g["rho_out"]) <= tol and abs(rl - g["rho_in"]) <= tol


def test_maxwell_equal_area_in_volume():
    """Independent route: the saturation pressure cuts equal areas of the P(v) loop, v = 1/rho."""
    for (a, b, T) in [(9 / 8, 1 / 3, 0.9), (2.0, 0.4, 0.85 * W.T_CRIT), (2.0, 0.4, 0.8 * W.T_CRIT)]:
        rv, rl = thermo.maxwell(T, a, b)
        Ps = thermo.pressure(rl, T, a, b)
        assert thermo.pressure(rv, T, a, b) == pytest.approx(Ps, rel=1e-10, abs=1e-13)
        vv, vl = 1 / rv, 1 / rl
        area, _ = integrate.quad(lambda v: thermo.pressure(1 / v, T, a, b), vl, vv, epsabs=0, epsrel=1e-13, limit=200)
        assert area == pytest.approx(Ps * (vv - vl), rel=1e-9)


def test_coexistence_is_universal_in_reduced_units():
    for t in (0.8, 0.9, 0.98):
        ref = None
        for a, b in ((9 / 8, 1 / 3), (2.0, 0.4), (0.7, 0.25)):
            Tc, rc = 8 * a / (27 * b), 1 / (3 * b)
            rv, rl = thermo.maxwell(t * Tc, a, b)
            red = np.array([rv / rc, rl / rc])
            if ref is None:
                ref = red
            np.testing.assert_allclose(red, ref, rtol=1e-9)


def test_workload_coexistence_table():
    for t, (rv, rl) in W.COEXISTENCE.items():
        mv, ml = thermo.maxwell(t * W.T_CRIT, W.EOS_A, W.EOS_B)
        assert abs(mv - rv) < 1e-6 and abs(ml - rl) < 1e-6


def test_surface_tension_printed_theory():
    """Sec. 4.2: theoretical sigma = 1.72e-4 and 1.40e-4 for K = 7.5e-6 and 5e-6 at T = 0.95
    (3 printed digits).  The first printed value, 1.96e-4 for K = 1e-5, contradicts
    sigma ~ sqrt(K) and the other two; the LB fit printed for it, 1.98e-4, matches."""
    g = GOLDEN["surface_tension_theory_T0.95"]
    sig = [thermo.surface_tension(g["T"], g["a"], g["b"], K) for K in g["K"]]
    for s, printed in zip(sig[1:], g["sigma"][1:]):
        assert abs(s - printed) <= 0.005e-4
    assert sig[0] == pytest.approx(math.sqrt(2) * sig[2], rel=1e-9)
    assert abs(sig[0] - GOLDEN["surface_tension_lb_T0.95"]["sigma"][0]) <= 0.005e-4
    assert abs(sig[0] - g["sigma"][0]) > 0.01e-4          # the printed 1.96e-4 is not reproduced


def test_surface_tension_two_routes():
    """Eq. (56): sigma = K int rho'^2 dz over the planar profile equals int sqrt(2 K omega) d rho."""
    T, a, b, K = 0.95, 9 / 8, 1 / 3, 1e-5
    z = np.linspace(-0.3, 0.3, 24001)
    prof = thermo.planar_profile(z, T, a, b, K)
    d = np.gradient(prof, z, edge_order=2)
    sig_z = K * integrate.simpson(d * d, x=z)
    assert sig_z == pytest.approx(thermo.surface_tension(T, a, b, K), rel=1e-6)
