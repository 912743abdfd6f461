"""Van der Waals equilibrium thermodynamics used to pin the FFT-LB oracle.

TEST INFRASTRUCTURE ONLY (see oracle/fftlb_oracle.py).

The fluid has P = rho T/(1 - b rho) - a rho^2 (Eq. (18) with parametrised
constants, R = 1).  This module computes, from the free energy of that fluid:

  * the coexistence densities by the Maxwell construction (Sec. 4.1 compares the
    simulated coexistence curve with it, Figs. 9 and 13);
  * the planar equilibrium interface of the square-gradient free energy
    psi(rho) + K |grad rho|^2 / 2, whose first integral is the interface-width
    integral of Sec. 4.1, Eqs. (51)-(53);
  * the surface tension sigma = K int (d rho/dz)^2 dz of Sec. 4.2, Eq. (56).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize


def free_energy_density(rho, T, a, b):
    """psi(rho) = rho T ln(rho/(1 - b rho)) - rho T - a rho^2, up to terms linear in rho;
    it gives P = rho psi' - psi = rho T/(1 - b rho) - a rho^2."""
    return rho * T * np.log(rho / (1.0 - b * rho)) - rho * T - a * rho * rho


def chemical_potential(rho, T, a, b):
    """mu = psi'(rho) = T ln(rho/(1 - b rho)) + T b rho/(1 - b rho) - 2 a rho."""
    return T * np.log(rho / (1.0 - b * rho)) + T * b * rho / (1.0 - b * rho) - 2.0 * a * rho


def pressure(rho, T, a, b):
    return rho * T / (1.0 - b * rho) - a * rho * rho


def spinodal(T, a, b):
    """Densities where dP/drho = 0 (T below the critical temperature 8a/27b)."""
    dp = lambda r: T / (1.0 - b * r) ** 2 - 2.0 * a * r
    rc = 1.0 / (3.0 * b)
    lo = optimize.brentq(dp, 1e-12, rc)
    hi = optimize.brentq(dp, rc, (1.0 - 1e-12) / b)
    return lo, hi


def maxwell(T, a, b):
    """Coexistence densities (rho_v, rho_l): equal pressure and equal chemical potential.

    For a trial pressure P between the spinodal pressures, rho_v(P) and rho_l(P) are the
    outer roots of P(rho) = P; the saturation pressure zeroes mu(rho_v) - mu(rho_l).
    """
    s_lo, s_hi = spinodal(T, a, b)
    p_min, p_max = pressure(s_hi, T, a, b), pressure(s_lo, T, a, b)

    def roots(P):
        # P(r) < r T, so P(P/(2T)) < P: a lower bracket for the vapour root.
        rv = optimize.brentq(lambda r: pressure(r, T, a, b) - P, 0.5 * P / T, s_lo,
                             xtol=1e-16, rtol=1e-15)
        rl = optimize.brentq(lambda r: pressure(r, T, a, b) - P, s_hi, (1.0 - 1e-14) / b,
                             xtol=1e-16, rtol=1e-15)
        return rv, rl

    def dmu(P):
        rv, rl = roots(P)
        return chemical_potential(rv, T, a, b) - chemical_potential(rl, T, a, b)

    lo = max(p_min, 0.0) + 1e-12 * abs(p_max)
    hi = p_max - 1e-14 * abs(p_max)
    Ps = optimize.brentq(dmu, lo, hi, xtol=1e-16, rtol=1e-15, maxiter=500)
    return roots(Ps)


def grand_potential(rho, T, a, b, rho_v, rho_l):
    """omega(rho) = psi - mu_s rho + P_s >= 0, zero at both coexistence densities."""
    mu_s = chemical_potential(rho_l, T, a, b)
    p_s = pressure(rho_l, T, a, b)
    return free_energy_density(rho, T, a, b) - mu_s * rho + p_s


_GL_X, _GL_W = np.polynomial.legendre.leggauss(40)


def grand_potential_accurate(rho, T, a, b, rho_v, rho_l):
    """omega(rho) without cancellation near the bulk densities:
    omega(rho) = int_{rho_s}^{rho} (rho - t) mu'(t) dt from the nearer coexistence density rho_s,
    with mu'(t) = T/(t (1 - b t)^2) - 2a (Gauss-Legendre quadrature)."""
    rho_s = rho_l if abs(rho - rho_l) < abs(rho - rho_v) else rho_v
    half = 0.5 * (rho - rho_s)
    t = rho_s + half * (_GL_X + 1.0)
    dmu = T / (t * (1.0 - b * t) ** 2) - 2.0 * a
    return float(half * np.sum(_GL_W * (rho - t) * dmu))


def planar_profile(s, T, a, b, K):
    """Equilibrium planar interface rho(s), vapour at s -> -inf, liquid at s -> +inf,
    centred where rho = (rho_v + rho_l)/2.

    Solves the first integral (K/2) rho'^2 = omega(rho), i.e. d rho/ds = sqrt(2 omega/K),
    which is the interface-width integral of Eqs. (51)-(53) written as an ODE.
    s is an increasing array of positions (same length unit as K's).
    """
    rho_v, rho_l = maxwell(T, a, b)
    mid = 0.5 * (rho_v + rho_l)
    s = np.asarray(s, dtype=np.float64)
    uniq, inverse = np.unique(s.ravel(), return_inverse=True)
    vals = np.empty_like(uniq)

    def speed(r):
        return math.sqrt(2.0 * max(grand_potential_accurate(r, T, a, b, rho_v, rho_l), 0.0) / K)

    # liquid side (s >= 0): d rho/ds = +speed, vapour side in t = -s: d rho/dt = -speed.
    # The sign factors make the bulk densities attracting fixed points of the ODE.
    branches = ((1.0, uniq >= 0.0, lambda t, y: [math.copysign(1.0, rho_l - y[0]) * speed(y[0])]),
                (-1.0, uniq < 0.0, lambda t, y: [-math.copysign(1.0, y[0] - rho_v) * speed(y[0])]))
    for sign, mask, rhs in branches:
        pts = sign * uniq[mask]                  # distances from the centre
        if pts.size == 0:
            continue
        order = np.argsort(pts)
        t_eval = pts[order]
        sol = integrate.solve_ivp(rhs, (0.0, t_eval[-1] + 1e-30), [mid], t_eval=t_eval,
                                  rtol=1e-13, atol=1e-16, method="DOP853")
        if sol.status != 0:
            raise RuntimeError("planar profile integration failed: " + sol.message)
        sub = np.empty_like(pts)
        sub[order] = sol.y[0]
        vals[mask] = sub
    return vals[inverse].reshape(s.shape)


def surface_tension(T, a, b, K):
    """sigma = K int (d rho/dz)^2 dz = int_{rho_v}^{rho_l} sqrt(2 K omega(rho)) d rho (Eq. (56))."""
    rho_v, rho_l = maxwell(T, a, b)
    val, _ = integrate.quad(
        lambda r: math.sqrt(max(2.0 * K * grand_potential(r, T, a, b, rho_v, rho_l), 0.0)),
        rho_v, rho_l, epsabs=0.0, epsrel=1e-12, limit=200)
    return val
