"""Exact solution of the one-dimensional Riemann problem of an ideal gas, for the modified
Sod shock tube the paper runs with the ideal-gas special case of the model (Sec. 3.6: the
Watari-Tsutahara model, a = b = K = q = 0, so that the force term vanishes).

TEST INFRASTRUCTURE ONLY (see oracle/fftlb_oracle.py).

The gas has p = rho T (R = 1).  The 33-velocity model in two dimensions carries the internal
energy rho T (Eq. (9): (1/2) sum |v - u|^2 f = rho T), i.e. e = T per unit mass, c_v = 1 and
gamma = (c_v + R) / c_v = 2.

The solution is the classical construction: the star-region pressure p* solves
f_L(p*) + f_R(p*) + (u_R - u_L) = 0, where f_K is the velocity jump across the K-wave
(a shock if p* > p_K, by the Rankine-Hugoniot conditions; a rarefaction otherwise, by the
isentropic relation p / rho^gamma = const and the Riemann invariant u +- 2c/(gamma - 1)); then
u* = (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2, and the fields at x/t follow the wave fan.
"""
from __future__ import annotations

import math

import numpy as np


def _wave_jump(p, rho_k, p_k, gamma):
    """Velocity change f_K(p) across the wave into state K and its derivative in p."""
    c_k = math.sqrt(gamma * p_k / rho_k)
    if p > p_k:  # shock: mass flux from the Rankine-Hugoniot conditions
        a_k = 2.0 / ((gamma + 1.0) * rho_k)
        b_k = (gamma - 1.0) / (gamma + 1.0) * p_k
        q = math.sqrt(a_k / (p + b_k))
        return (p - p_k) * q, q * (1.0 - 0.5 * (p - p_k) / (p + b_k))
    # rarefaction: isentropic, Riemann invariant
    e = (gamma - 1.0) / (2.0 * gamma)
    r = (p / p_k) ** e
    return 2.0 * c_k / (gamma - 1.0) * (r - 1.0), (p / p_k) ** (e - 1.0) / (rho_k * c_k)


def star_state(rho_l, u_l, p_l, rho_r, u_r, p_r, gamma):
    """(p*, u*) of the Riemann problem by Newton's method on f_L + f_R + du = 0."""
    du = u_r - u_l
    p = max(1e-12, 0.5 * (p_l + p_r))
    for _ in range(100):
        fl, dfl = _wave_jump(p, rho_l, p_l, gamma)
        fr, dfr = _wave_jump(p, rho_r, p_r, gamma)
        g = fl + fr + du
        step = g / (dfl + dfr)
        p_new = max(1e-14, p - step)
        if abs(p_new - p) <= 1e-15 * (p_new + p):
            p = p_new
            break
        p = p_new
    fl, _ = _wave_jump(p, rho_l, p_l, gamma)
    fr, _ = _wave_jump(p, rho_r, p_r, gamma)
    return p, 0.5 * (u_l + u_r) + 0.5 * (fr - fl)


def star_densities(rho_l, p_l, rho_r, p_r, p_star, gamma):
    """Densities left and right of the contact: shock adiabat or isentrope."""
    def side(rho_k, p_k):
        if p_star > p_k:
            g = (gamma - 1.0) / (gamma + 1.0)
            return rho_k * (p_star / p_k + g) / (g * p_star / p_k + 1.0)
        return rho_k * (p_star / p_k) ** (1.0 / gamma)
    return side(rho_l, p_l), side(rho_r, p_r)


def sample(xi, rho_l, u_l, p_l, rho_r, u_r, p_r, gamma):
    """(rho, u, p) at the similarity coordinate xi = x / t (arrays)."""
    p_s, u_s = star_state(rho_l, u_l, p_l, rho_r, u_r, p_r, gamma)
    rho_sl, rho_sr = star_densities(rho_l, p_l, rho_r, p_r, p_s, gamma)
    c_l = math.sqrt(gamma * p_l / rho_l)
    c_r = math.sqrt(gamma * p_r / rho_r)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for i, s in np.ndenumerate(xi):
        if s <= u_s:  # left of the contact
            if p_s > p_l:  # left shock
                S = u_l - c_l * math.sqrt((gamma + 1.0) / (2.0 * gamma) * p_s / p_l + (gamma - 1.0) / (2.0 * gamma))
                vals = (rho_l, u_l, p_l) if s < S else (rho_sl, u_s, p_s)
            else:  # left rarefaction: head u_l - c_l, tail u* - c*_l
                c_sl = c_l * (p_s / p_l) ** ((gamma - 1.0) / (2.0 * gamma))
                if s < u_l - c_l:
                    vals = (rho_l, u_l, p_l)
                elif s > u_s - c_sl:
                    vals = (rho_sl, u_s, p_s)
                else:
                    uu = 2.0 / (gamma + 1.0) * (c_l + 0.5 * (gamma - 1.0) * u_l + s)
                    cc = 2.0 / (gamma + 1.0) * (c_l + 0.5 * (gamma - 1.0) * (u_l - s))
                    rr = rho_l * (cc / c_l) ** (2.0 / (gamma - 1.0))
                    vals = (rr, uu, p_l * (cc / c_l) ** (2.0 * gamma / (gamma - 1.0)))
        else:  # right of the contact
            if p_s > p_r:  # right shock
                S = u_r + c_r * math.sqrt((gamma + 1.0) / (2.0 * gamma) * p_s / p_r + (gamma - 1.0) / (2.0 * gamma))
                vals = (rho_r, u_r, p_r) if s > S else (rho_sr, u_s, p_s)
            else:  # right rarefaction
                c_sr = c_r * (p_s / p_r) ** ((gamma - 1.0) / (2.0 * gamma))
                if s > u_r + c_r:
                    vals = (rho_r, u_r, p_r)
                elif s < u_s + c_sr:
                    vals = (rho_sr, u_s, p_s)
                else:
                    uu = 2.0 / (gamma + 1.0) * (-c_r + 0.5 * (gamma - 1.0) * u_r + s)
                    cc = 2.0 / (gamma + 1.0) * (c_r - 0.5 * (gamma - 1.0) * (u_r - s))
                    rr = rho_r * (cc / c_r) ** (2.0 / (gamma - 1.0))
                    vals = (rr, uu, p_r * (cc / c_r) ** (2.0 * gamma / (gamma - 1.0)))
        rho[i], u[i], p[i] = vals
    return rho, u, p
