"""FP64 CPU oracle of one FFT-LB time step of the thermal van der Waals model.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow reference that the
HIP path is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the library and its Python binding
never do, and it shares no code, tables or constants with them.

Everything here is written from the paper (Gan, Xu, Zhang, Li, "FFT-LB modeling
of thermal liquid-vapor systems"); equation numbers follow the compiled paper.

  * Sec. 2.1  Watari-Tsutahara 33-velocity model: velocities Eq. (1), equilibrium
              Eq. (3), weights Eqs. (4)-(6), moments Eqs. (7)-(9).
  * Sec. 2.2  Gonnella-Lamura-Sofonea force term: kinetic equation Eq. (10),
              force Eq. (11), total energy Eq. (17), EOS Eq. (18), pressure
              tensor Eq. (19), coefficients Eqs. (20)-(23).
  * Sec. 3    forward-Euler update in the form of Eq. (24); every spatial
              derivative by the windowed FFT: transform pair Eqs. (40)-(41),
              derivative theorem Eq. (42), windowed wavenumbers Eqs. (43)-(47).

Readings of points the paper leaves open (each one is listed in the design doc):
  R1  the Nyquist wavenumber of a first-derivative operator is set to zero;
  R2  second derivatives are compositions of first derivatives;
  R3  divergences are taken of the product fields (conservative form, as printed);
  R4  the same windowed operator (order m) is used for every derivative;
  R5  in 2D the window acts per axis on that axis' wavenumber;
  R6  unsplit forward Euler with every right-hand-side term at level n;
  R7  moments are taken of f (they equal those of f^eq by construction);
  R8  EOS constants are parameters: P^w = rho T/(1 - b rho) - a rho^2 and the
      9/8 of Eqs. (17) and (22) becomes a (the paper's a = 9/8, b = 1/3);
  R10 the initial distribution is f^eq(rho0, u0, T0);
  R23 the one-dimensional finite-difference schemes of Sec. 3.1 (LW, MLW1, MLW2) act along
      x with c = v_x dt/dx and along y with c = v_y dt/dy, and their updates add;
  R26 flux limiter: where g_{J+1} = g_J the limited term of the flux is zero (theta undefined);
  R24 with the NPS stencils the Laplacian of the pressure tensor is the nine-point one, the
      derivatives of theta are compositions of first derivatives, and the convection term is
      v_x D_x f + v_y D_y f with the nine-point first derivatives.

Array layout: fields are [ny, nx] (x fastest); distributions are [33, ny, nx]
with q = 0 the rest particle and q = 1 + 8(k-1) + (i-1) for speed group k and
direction i.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.fft as sfft

# Sec. 2.1, text after Eq. (1): the four speeds of the velocity groups.
SPEEDS = (1.00, 1.90, 2.90, 4.30)

# Eqs. (44)-(47): coefficients of sin^(2j+1)(k dx/2) in the truncated series of
# arcsin(sin(k dx/2)); k_m keeps the first m of them.
ARCSIN_COEFFS = (1.0, 1.0 / 6.0, 3.0 / 40.0, 5.0 / 112.0)

Q = 33


@dataclasses.dataclass(frozen=True)
class Params:
    """Model and discretisation parameters (Sec. 2.2 and the parameter list of Sec. 3.5).

    The paper's values are dx = dy = 1/256, dt = 1e-5, tau = 1e-2, K = 1e-5,
    H = 0, zeta = 0, q = -0.004 and the k4 window (m = 4); its EOS is a = 9/8,
    b = 1/3.  m = 0 selects the exact wavenumber k.  conv = 0 takes the convection term
    with the derivative operator of m; LAX_WENDROFF, MLW1, MLW2 or FLUX_LIMITER with that
    finite-difference scheme of Sec. 3.1.
    """
    dx: float = 1.0 / 256.0
    dy: float = 1.0 / 256.0
    dt: float = 1e-5
    tau: float = 1e-2
    K: float = 1e-5
    H: float = 0.0
    zeta: float = 0.0
    q: float = -0.004
    a: float = 9.0 / 8.0
    b: float = 1.0 / 3.0
    m: int = 4
    conv: int = 0


def critical_point(a: float, b: float):
    """Critical temperature and density of P = rho T/(1 - b rho) - a rho^2 (R = 1)."""
    return 8.0 * a / (27.0 * b), 1.0 / (3.0 * b)


# ----------------------------------------------------------------------------
# Sec. 2.1: discrete velocities, weights, equilibrium, moments
# ----------------------------------------------------------------------------

def velocities() -> np.ndarray:
    """Eq. (1): v_0 = 0 and v_ki = v_k (cos((i-1) pi/4), sin((i-1) pi/4)).

    The cosines and sines of multiples of pi/4 are written as their exact values
    (0, +-1, +-sqrt(2)/2) so that axis-aligned velocities have exact zeros.
    """
    r = math.sqrt(0.5)
    cos8 = (1.0, r, 0.0, -r, -1.0, -r, 0.0, r)
    sin8 = (0.0, r, 1.0, r, 0.0, -r, -1.0, -r)
    v = np.zeros((Q, 2))
    for k in range(4):
        for i in range(8):
            v[1 + 8 * k + i, 0] = SPEEDS[k] * cos8[i]
            v[1 + 8 * k + i, 1] = SPEEDS[k] * sin8[i]
    return v


def weights(T):
    """Eqs. (4)-(6): weights F_1..F_4 of the speed groups and F_0 of the rest particle.

    F_k = [48 T^4 - 6 S1 T^3 + S2 T^2 - S3 T / 4] / [v_k^2 prod_l (v_k^2 - v_{k+l}^2)]
    with S1, S2, S3 the elementary symmetric sums of v_{k+1}^2, v_{k+2}^2, v_{k+3}^2
    and the cyclic index {k+l} of Eq. (6).  F_0 = 1 - 8 (F_1 + F_2 + F_3 + F_4).
    Returns (F0, [F1, F2, F3, F4]); T may be a scalar or an array.
    """
    s = [v * v for v in SPEEDS]
    F = []
    for k in range(4):
        s1, s2, s3 = s[(k + 1) % 4], s[(k + 2) % 4], s[(k + 3) % 4]
        num = (48.0 * T**4 - 6.0 * (s1 + s2 + s3) * T**3
               + (s1 * s2 + s2 * s3 + s3 * s1) * T**2 - s1 * s2 * s3 * T / 4.0)
        den = s[k] * (s[k] - s1) * (s[k] - s2) * (s[k] - s3)
        F.append(num / den)
    F0 = 1.0 - 8.0 * (F[0] + F[1] + F[2] + F[3])
    return F0, F


def feq(rho, ux, uy, T):
    """Eq. (3): fourth-order expansion of the local Maxwellian in u, times rho F_k.

    f^eq = rho F_k [ (1 - u^2/2T + u^4/8T^2) + (v.u/T)(1 - u^2/2T)
                     + ((v.u)^2/2T^2)(1 - u^2/2T) + (v.u)^3/6T^3 + (v.u)^4/24T^4 ].
    """
    rho, ux, uy, T = (np.asarray(x, dtype=np.float64) for x in (rho, ux, uy, T))
    v = velocities()
    F0, F = weights(T)
    u2 = ux * ux + uy * uy
    g = 1.0 - u2 / (2.0 * T)
    base = g + u2 * u2 / (8.0 * T * T)
    out = np.empty((Q,) + rho.shape)
    out[0] = rho * F0 * base
    for q in range(1, Q):
        k = (q - 1) // 8
        vu = v[q, 0] * ux + v[q, 1] * uy
        poly = (base + vu / T * g + vu * vu / (2.0 * T * T) * g
                + vu**3 / (6.0 * T**3) + vu**4 / (24.0 * T**4))
        out[q] = rho * F[k] * poly
    return out


def moments(f):
    """Eqs. (7)-(9) evaluated on f: rho = sum f, rho u = sum v f, rho T = sum |v - u|^2 f / 2."""
    f = np.asarray(f, dtype=np.float64)
    v = velocities()
    rho = f.sum(axis=0)
    ux = np.tensordot(v[:, 0], f, axes=1) / rho
    uy = np.tensordot(v[:, 1], f, axes=1) / rho
    e = np.zeros_like(rho)
    for q in range(Q):
        cx = v[q, 0] - ux
        cy = v[q, 1] - uy
        e += 0.5 * (cx * cx + cy * cy) * f[q]
    return rho, ux, uy, e / rho


# ----------------------------------------------------------------------------
# Sec. 3.6: windowed-FFT derivative operator
# ----------------------------------------------------------------------------

def wavenumbers(n: int, delta: float) -> np.ndarray:
    """k = 2 pi n' / L for the FFT ordering n' = 0..n/2-1, -n/2..-1 (Eq. (41)), L = n delta."""
    return 2.0 * np.pi * np.fft.fftfreq(n, d=delta)


# Derivative order m = CENTRAL_DIFFERENCE selects the second-order central difference of
# Sec. 3.1, (g[J+1] - g[J-1]) / (2 delta), for every derivative (the CD + CD comparison scheme of
# the paper's Fig. 2); the oracle applies it as that stencil in real space.
CENTRAL_DIFFERENCE = 5

# Derivative order m = NPS selects the nine-point stencils of Sec. 3.1 (the NPS scheme) for every
# derivative and for the convection term: the first derivative with weights A (the row through
# the node) and B (the two rows beside it), 2A + 4B = 1, B = 1/12; the Laplacian with weights E
# (edges) and F (corners), E + 2F = 1, F = 1/6.  Second derivatives other than the Laplacian
# are compositions of the first ones (R2).  The paper uses dx = dy with these stencils.
NPS = 6
NPS_B = 1.0 / 12.0
NPS_A = (1.0 - 4.0 * NPS_B) / 2.0
NPS_F = 1.0 / 6.0
NPS_E = 1.0 - 2.0 * NPS_F


def kappa(n: int, delta: float, m: int) -> np.ndarray:
    """Windowed wavenumber k_m of Eqs. (44)-(47); m = 0 is the exact k.

    k_m = (2/delta) sum_{j<m} c_j sin^(2j+1)(k delta / 2) with c = (1, 1/6, 3/40, 5/112).
    The Nyquist entry n' = -n/2 is zero (reading R1): it keeps the operator real.
    m = CENTRAL_DIFFERENCE: the symbol of the central-difference stencil, sin(k delta) / delta
    (the stencil multiplies the mode exp(i k x) by (e^(i k delta) - e^(-i k delta)) / (2 delta)).
    """
    if n % 2:
        raise ValueError("grid size must be even")
    k = wavenumbers(n, delta)
    if m == 0:
        kap = k.copy()
    elif m == CENTRAL_DIFFERENCE:
        kap = np.sin(k * delta) / delta
    else:
        if not 1 <= m <= len(ARCSIN_COEFFS):
            raise ValueError("window order m must be 0..4")
        s = np.sin(0.5 * k * delta)
        kap = np.zeros(n)
        for j in range(m):
            kap += ARCSIN_COEFFS[j] * s ** (2 * j + 1)
        kap *= 2.0 / delta
    kap[n // 2] = 0.0
    return kap


def fft2(g, workers=None):
    """Forward 2D DFT with kernel exp(-i k.x), Eq. (40) without the dx dy factor."""
    return sfft.fft2(g, workers=workers)


def ifft2(G, workers=None):
    """Inverse 2D DFT with the 1/(nx ny) factor, Eq. (41) (the dx dy and 1/L factors cancel)."""
    return sfft.ifft2(G, workers=workers)


class Deriv:
    """The windowed-FFT first-derivative operators D_x, D_y on one periodic grid.

    D_alpha g = Re IFFT2[ i kappa_m(k_alpha) FFT2(g) ]  (Eq. (42) with k -> k_m; R4, R5).
    With m = CENTRAL_DIFFERENCE: the stencil (g[J+1] - g[J-1]) / (2 delta) along alpha (Sec. 3.1).
    """

    def __init__(self, ny: int, nx: int, p: Params, workers=None):
        self.cd = p.m == CENTRAL_DIFFERENCE
        self.nps = p.m == NPS
        self.stencil = self.cd or self.nps
        if self.nps and p.dx != p.dy:
            raise ValueError("the NPS stencils need dx = dy")
        self.dx, self.dy = p.dx, p.dy
        if not self.stencil:
            self.kx = kappa(nx, p.dx, p.m)[None, :]
            self.ky = kappa(ny, p.dy, p.m)[:, None]
        self.workers = workers

    def spectrum(self, g):
        return fft2(g, self.workers)

    def from_spectrum(self, G):
        return ifft2(G, self.workers).real

    def x(self, g):
        if self.cd:
            return (np.roll(g, -1, axis=1) - np.roll(g, 1, axis=1)) / (2.0 * self.dx)
        if self.nps:
            return _nps_first(g, 1, 0) / self.dx
        return self.from_spectrum(1j * self.kx * self.spectrum(g))

    def y(self, g):
        if self.cd:
            return (np.roll(g, -1, axis=0) - np.roll(g, 1, axis=0)) / (2.0 * self.dy)
        if self.nps:
            return _nps_first(g, 0, 1) / self.dy
        return self.from_spectrum(1j * self.ky * self.spectrum(g))

    def laplacian(self, g):
        """The nine-point Laplacian with the NPS stencils; otherwise D_x D_x g + D_y D_y g (R2)."""
        if self.nps:
            return _nps_laplacian(g) / (self.dx * self.dx)
        return self.x(self.x(g)) + self.y(self.y(g))


def _nps_first(g, along, across):
    """Nine-point first difference (times the spacing) along axis `along`: A times the
    difference of the two neighbours on the node's own line, plus B times the differences on
    the two lines beside it (offset by one node along `across`)."""
    diff = np.roll(g, -1, axis=along) - np.roll(g, 1, axis=along)
    return NPS_A * diff + NPS_B * (np.roll(diff, -1, axis=across) + np.roll(diff, 1, axis=across))


def _nps_laplacian(g):
    """Nine-point Laplacian (times the spacing squared): E times the four edge neighbours, F
    times the four corner neighbours, -4 (E + F) times the node."""
    edges = np.roll(g, 1, 0) + np.roll(g, -1, 0) + np.roll(g, 1, 1) + np.roll(g, -1, 1)
    corners = sum(np.roll(np.roll(g, a, 0), b, 1) for a in (1, -1) for b in (1, -1))
    return NPS_E * edges + NPS_F * corners - 4.0 * (NPS_E + NPS_F) * g


# Sec. 3.1: finite-difference schemes of the convection term, compared in the paper's
# Fig. 2 (with the central difference for the force): Lax-Wendroff, Eq. (ML-); MLW1 adds the
# discretised dispersion term R3, Eq. (R3); MLW2 adds R3 and the dissipation term R4, Eq. (R4=).
LAX_WENDROFF, MLW1, MLW2 = 1, 2, 3
# The flux-limiter scheme of Sec. 3.1: the convection of each population along its
# characteristic line (its own lattice direction), with the MCD limiter.
FLUX_LIMITER = 4


def fd_convection_update(g, c, axis, scheme):
    """Change of g at every node J in one forward-Euler step from the convection along one
    axis, as the schemes of Sec. 3.1 write it, with CFL number c = v_alpha dt / d_alpha and
    the periodic neighbours J-2..J+2 along `axis`:
      LW  (Eq. (ML-)): -(c/2)(g[J+1] - g[J-1]) + (c^2/2)(g[J+1] - 2 g[J] + g[J-1])
      R3  (Eq. (R3)):  c (1 - c^2)/12 (g[J+2] - 2 g[J+1] + 2 g[J-1] - g[J-2])     (MLW1, MLW2)
      R4  (Eq. (R4=)): c^2 (1 - c^2)/8 (g[J+2] - 4 g[J+1] + 6 g[J] - 4 g[J-1] + g[J-2])  (MLW2)
    """
    if scheme not in (LAX_WENDROFF, MLW1, MLW2):
        raise ValueError("scheme must be LAX_WENDROFF, MLW1 or MLW2")
    gp1 = np.roll(g, -1, axis=axis)   # g[J+1] at J
    gm1 = np.roll(g, 1, axis=axis)    # g[J-1]
    du = -0.5 * c * (gp1 - gm1) + 0.5 * c * c * (gp1 - 2.0 * g + gm1)
    if scheme >= MLW1:
        gp2 = np.roll(g, -2, axis=axis)
        gm2 = np.roll(g, 2, axis=axis)
        du = du + c * (1.0 - c * c) / 12.0 * (gp2 - 2.0 * gp1 + 2.0 * gm1 - gm2)
        if scheme >= MLW2:
            du = du + c * c * (1.0 - c * c) / 8.0 * (gp2 - 4.0 * gp1 + 6.0 * g - 4.0 * gm1 + gm2)
    return du


def mcd_limiter(theta):
    """psi(theta) of the monotonized central-difference limiter (Sec. 3.1): 0 for theta <= 0,
    2 theta up to 1/3, (1 + theta)/2 up to 3, 2 beyond."""
    theta = np.asarray(theta, dtype=np.float64)
    return np.where(theta <= 0.0, 0.0,
                    np.where(theta <= 1.0 / 3.0, 2.0 * theta, np.where(theta <= 3.0, 0.5 * (1.0 + theta), 2.0)))


def _along(g, e, n):
    """g at J + n e on the periodic grid (e = (ex, ey) a lattice step; arrays are [y, x])."""
    return np.roll(np.roll(g, -n * e[1], axis=0), -n * e[0], axis=1)


def fl_convection_update(g, c, e, limiter=mcd_limiter):
    """Change of g in one forward-Euler step from its convection along the characteristic line
    through every node (Sec. 3.1, Eq. (FL)): J +- 1 are the neighbours at J +- e, c the CFL number
    v_k dt / (A_i dr) of the line.  With theta_J = (g_J - g_{J-1}) / (g_{J+1} - g_J),
      F_{J+1/2} = g_J + (1 - c)/2 (g_{J+1} - g_J) psi(theta_J),   F_{J-1/2} = F_{(J-1)+1/2},
    and the change is -c (F_{J+1/2} - F_{J-1/2}).  Where g_{J+1} = g_J, theta is undefined and
    the limited term (g_{J+1} - g_J) psi vanishes with its factor (reading R26)."""
    def flux(gm, g0, gp):
        den = gp - g0
        safe = np.where(den != 0.0, den, 1.0)
        theta = np.where(den != 0.0, (g0 - gm) / safe, 0.0)
        return g0 + 0.5 * (1.0 - c) * den * limiter(theta)
    gp1, gm1, gm2 = _along(g, e, 1), _along(g, e, -1), _along(g, e, -2)
    return -c * (flux(gm1, g, gp1) - flux(gm2, gm1, g))


def characteristic(v):
    """Lattice step e and factor A_i of a velocity of Eq. (1): e = the signs of its components,
    A_i = 1 along an axis, sqrt(2) along a diagonal (Sec. 3.1)."""
    ex = int(np.sign(round(v[0], 9)))
    ey = int(np.sign(round(v[1], 9)))
    return (ex, ey), (math.sqrt(2.0) if ex and ey else 1.0)


def convection(f, v, D: Deriv, p: Params | None = None):
    """Convection term v_q . grad f_q by windowed FFT (Sec. 3.6, Fig. 3 flow chart).

    By linearity of Eq. (42), FT[v.grad f] = i (v_x k_x + v_y k_y) FT[f]; one
    forward and one inverse transform per moving population.  C_0 = 0.  With the central
    difference or the NPS stencils: v_x D_x f + v_y D_y f by the stencil (Sec. 3.1).
    With a finite-difference scheme (p.conv): the updates of fd_convection_update along x
    (c = v_x dt/dx) and along y (c = v_y dt/dy) added (reading R23), returned as the term C
    that the step subtracts times dt: C = -(du_x + du_y) / dt.
    """
    out = np.zeros_like(f)
    scheme = p.conv if p is not None else 0
    if scheme == FLUX_LIMITER and p.dx != p.dy:
        raise ValueError("the flux-limiter scheme needs dx = dy")
    for q in range(1, f.shape[0]):
        if scheme == FLUX_LIMITER:
            e, A = characteristic(v[q])
            speed = math.hypot(v[q, 0], v[q, 1])
            out[q] = -fl_convection_update(f[q], speed * p.dt / (A * p.dx), e) / p.dt
            continue
        if scheme:
            du = (fd_convection_update(f[q], v[q, 0] * p.dt / p.dx, 1, scheme)
                  + fd_convection_update(f[q], v[q, 1] * p.dt / p.dy, 0, scheme))
            out[q] = -du / p.dt
            continue
        if D.stencil:
            out[q] = v[q, 0] * D.x(f[q]) + v[q, 1] * D.y(f[q])
            continue
        mult = 1j * (v[q, 0] * D.kx + v[q, 1] * D.ky)
        out[q] = D.from_spectrum(mult * D.spectrum(f[q]))
    return out


# ----------------------------------------------------------------------------
# Sec. 2.2: van der Waals force
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Force:
    A: np.ndarray
    Bx: np.ndarray
    By: np.ndarray
    C: np.ndarray
    Cq: np.ndarray
    # stage-1 derivatives, kept for diagnostics and tests
    rx: np.ndarray
    ry: np.ndarray
    lap: np.ndarray
    theta: np.ndarray
    Pw: np.ndarray
    Lxx: np.ndarray
    Lxy: np.ndarray
    Lyy: np.ndarray


def pressure_vdw(rho, T, p: Params):
    """Eq. (18) with parametrised constants (R8): P^w = rho T/(1 - b rho) - a rho^2."""
    return rho * T / (1.0 - p.b * rho) - p.a * rho * rho


def force_coefficients(rho, ux, uy, T, p: Params, D: Deriv) -> Force:
    """Coefficients of the force term, Eqs. (19)-(23), with every derivative by D.

    Lambda_ab = M d_a rho d_b rho - [rho T grad rho . grad(M/T)] delta_ab
                - M (rho lap rho + |grad rho|^2 / 2) delta_ab,      M = K + H T;
    grad(M/T) = -K grad T / T^2 for any H, so the bracket is -rho K grad rho.grad T / T.
    B_a  = [d_a(P^w - rho T) + d_b Lambda_ab - d_a(zeta theta)] / (rho T)   (Eq. (21), R3)
    C    = {(P^w - rho T) theta + Lambda_ab d_a u_b - zeta theta^2 + a rho^2 theta
            + K[-|grad rho|^2 theta / 2 - rho grad rho.grad theta
                - d_g rho d_g u_a d_a rho]} / (2 rho T^2)                    (Eq. (22), R8)
    C_q  = d_a[2 q rho T d_a T] / (2 rho T^2)                              (Eq. (23), R3)
    A    = -2 (C + C_q) T                                                  (Eq. (20))
    """
    rx, ry = D.x(rho), D.y(rho)
    lap = D.laplacian(rho) if D.nps else D.x(rx) + D.y(ry)   # R2 (NPS: the nine-point Laplacian)
    dxux, dyux = D.x(ux), D.y(ux)
    dxuy, dyuy = D.x(uy), D.y(uy)
    theta = dxux + dyuy
    thx, thy = D.x(theta), D.y(theta)             # R2
    Tx, Ty = D.x(T), D.y(T)

    M = p.K + p.H * T
    Pw = pressure_vdw(rho, T, p)
    grad2 = rx * rx + ry * ry
    iso = rho * p.K * (rx * Tx + ry * Ty) / T - M * (rho * lap + 0.5 * grad2)
    Lxx = M * rx * rx + iso
    Lyy = M * ry * ry + iso
    Lxy = M * rx * ry

    # Eq. (21): every divergence of a product field is formed after the product (R3).
    nonideal = Pw - rho * T
    bulk = p.zeta * theta
    Bx = (D.x(nonideal) + D.x(Lxx) + D.y(Lxy) - D.x(bulk)) / (rho * T)
    By = (D.y(nonideal) + D.x(Lxy) + D.y(Lyy) - D.y(bulk)) / (rho * T)

    # Eq. (22)
    lam_du = Lxx * dxux + Lxy * dxuy + Lxy * dyux + Lyy * dyuy
    grad_rho_grad_theta = rx * thx + ry * thy
    cubic = rx * (dxux * rx + dxuy * ry) + ry * (dyux * rx + dyuy * ry)
    C = (nonideal * theta + lam_du - bulk * theta + p.a * rho * rho * theta
         + p.K * (-0.5 * grad2 * theta - rho * grad_rho_grad_theta - cubic)) / (2.0 * rho * T * T)

    # Eq. (23)
    gx = 2.0 * p.q * rho * T * Tx
    gy = 2.0 * p.q * rho * T * Ty
    Cq = (D.x(gx) + D.y(gy)) / (2.0 * rho * T * T)

    A = -2.0 * (C + Cq) * T
    return Force(A=A, Bx=Bx, By=By, C=C, Cq=Cq, rx=rx, ry=ry, lap=lap,
                 theta=theta, Pw=Pw, Lxx=Lxx, Lxy=Lxy, Lyy=Lyy)


def force_term(fe, ux, uy, fc: Force):
    """Eq. (11): I_q = -[A + B.(v_q - u) + (C + C_q) |v_q - u|^2] f^eq_q."""
    v = velocities()
    out = np.empty_like(fe)
    for q in range(Q):
        cx = v[q, 0] - ux
        cy = v[q, 1] - uy
        out[q] = -(fc.A + fc.Bx * cx + fc.By * cy + (fc.C + fc.Cq) * (cx * cx + cy * cy)) * fe[q]
    return out


# ----------------------------------------------------------------------------
# Sec. 3: the time step
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class StepParts:
    f_next: np.ndarray
    rho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    T: np.ndarray
    feq: np.ndarray
    conv: np.ndarray
    I: np.ndarray
    force: Force


def step_parts(f, p: Params, workers=None) -> StepParts:
    """One explicit step (R6) of Eq. (10), in the conservative form of Eq. (24):

    f^{n+1}_q = f^n_q - dt v_q.grad f^n_q - (dt/tau)(f^n_q - f^eq_q) + dt I_q.
    tau = inf switches the collision off.
    """
    f = np.asarray(f, dtype=np.float64)
    ny, nx = f.shape[1:]
    D = Deriv(ny, nx, p, workers)
    rho, ux, uy, T = moments(f)
    fc = force_coefficients(rho, ux, uy, T, p, D)
    fe = feq(rho, ux, uy, T)
    conv = convection(f, velocities(), D, p)
    I = force_term(fe, ux, uy, fc)
    relax = 0.0 if math.isinf(p.tau) else p.dt / p.tau
    f_next = f - p.dt * conv - relax * (f - fe) + p.dt * I
    return StepParts(f_next, rho, ux, uy, T, fe, conv, I, fc)


def step(f, p: Params, workers=None):
    return step_parts(f, p, workers).f_next


def run(f, p: Params, nsteps: int, workers=None):
    for _ in range(nsteps):
        f = step(f, p, workers)
    return f


def init_distribution(rho0, ux0, uy0, T0):
    """Reading R10: f^0 = f^eq(rho0, u0, T0)."""
    return feq(rho0, ux0, uy0, T0)


# ----------------------------------------------------------------------------
# Global diagnostics
# ----------------------------------------------------------------------------

def total_energy_density(rho, ux, uy, T, rx, ry, p: Params):
    """Eq. (17) with 9/8 -> a (R8): e_T = rho T - a rho^2 + K |grad rho|^2 / 2 + rho u^2 / 2."""
    return rho * T - p.a * rho * rho + 0.5 * p.K * (rx * rx + ry * ry) + 0.5 * rho * (ux * ux + uy * uy)


def globals_of(f, p: Params, workers=None):
    """Mass, momentum and total energy (Eq. (17)) summed over the grid times dx dy,
    plus max |u|.  Returned as a dict of Python floats."""
    f = np.asarray(f, dtype=np.float64)
    ny, nx = f.shape[1:]
    D = Deriv(ny, nx, p, workers)
    rho, ux, uy, T = moments(f)
    rx, ry = D.x(rho), D.y(rho)
    cell = p.dx * p.dy
    e = total_energy_density(rho, ux, uy, T, rx, ry, p)
    return dict(mass=float(rho.sum() * cell), px=float((rho * ux).sum() * cell),
                py=float((rho * uy).sum() * cell), energy=float(e.sum() * cell),
                umax=float(np.sqrt(ux * ux + uy * uy).max()))


def fields_energy(rho, ux, uy, T, p: Params, workers=None) -> float:
    """Total energy of macroscopic fields, sum e_T dx dy with e_T of Eq. (17) and the
    windowed derivatives of rho (the energy of the state f^eq(rho, u, T))."""
    rho, ux, uy, T = (np.asarray(a, dtype=np.float64) for a in (rho, ux, uy, T))
    D = Deriv(rho.shape[0], rho.shape[1], p, workers)
    e = total_energy_density(rho, ux, uy, T, D.x(rho), D.y(rho), p)
    return float(e.sum() * p.dx * p.dy)


def match_energy(rho, ux, uy, T, energy: float, p: Params, workers=None):
    """Temperature field shifted uniformly so that the fields carry the total energy
    `energy`.  In Eq. (17) the temperature enters e_T only through rho T, so a uniform
    shift dT changes the total by dT sum rho dx dy (the mass): dT = (energy - E) / mass.
    Returns T + dT (density and velocity are left as they are)."""
    rho = np.asarray(rho, dtype=np.float64)
    mass = float(rho.sum() * p.dx * p.dy)
    dT = (energy - fields_energy(rho, ux, uy, T, p, workers)) / mass
    return np.asarray(T, dtype=np.float64) + dT


def residual(conv, p: Params) -> float:
    """dt max_sites |sum_q C_q|: the density change per step carried by convection
    (the collision and the force conserve mass at every site, Eqs. (7), (11))."""
    return float(p.dt * np.abs(conv.sum(axis=0)).max())


def momentum_residual(f, p: Params) -> float:
    """dt max_sites |D_x(rho u_x) + D_y(rho u_y)| of the state f: the same quantity as
    residual() of the next step's convection terms, because the windowed derivative is
    linear and sum_q v_q f_q = rho u (Eq. (8))."""
    rho, ux, uy, _ = moments(f)
    D = Deriv(f.shape[1], f.shape[2], p)
    return float(p.dt * np.abs(D.x(rho * ux) + D.y(rho * uy)).max())
