"""Seeded synthetic initial conditions for the FFT-LB thermal liquid-vapour step.

This module only draws and shapes initial fields; it holds none of the method's
arithmetic.  Both the HIP path's tests and the FP64 oracle's tests take their
inputs from here, so the two sides always start from the same numbers.

Every generator builds the fields in float64 and returns them rounded to
float32 (the GPU precision); callers that feed the oracle promote those float32
values back to float64, so both sides see bit-identical initial data.

The workloads mirror the paper's own set-ups: a liquid slab between two planar
interfaces (Sec. 4.1, Eq. (50)), a droplet (Sec. 4.2, Eq. (54)) and a quench from
a uniform density with small random perturbations (the phase-separation test of
Sec. 3.5, Eq. (39)).  No dataset is involved.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Model parameters adopted from the paper's parameter list (Sec. 3.5):
# dx = dy = 1/256, dt = 1e-5, tau = 1e-2, K = 1e-5, H = 0, zeta = 0, q = -0.004,
# and the k4 window (Sec. 4.1).  The benchmark fluid uses a = 2, b = 0.4.
PAPER_PARAMS = dict(dx=1.0 / 256.0, dy=1.0 / 256.0, dt=1e-5, tau=1e-2, K=1e-5, H=0.0,
                    zeta=0.0, q=-0.004, m=4)
EOS_A, EOS_B = 2.0, 0.4
T_CRIT = 8.0 * EOS_A / (27.0 * EOS_B)   # 1.481481...
RHO_CRIT = 1.0 / (3.0 * EOS_B)          # 0.833333...

# Maxwell-construction coexistence densities (rho_v, rho_l) of the a = 2, b = 0.4
# fluid at T / T_crit; used only to shape initial profiles.  A CPU test re-derives
# them with the oracle's Maxwell construction.
COEXISTENCE = {
    0.80: (0.199722, 1.610588),
    0.81: (0.211738, 1.590877),
    0.82: (0.224370, 1.570606),
    0.83: (0.237663, 1.549730),
    0.84: (0.251667, 1.528198),
    0.85: (0.266442, 1.505950),
    0.86: (0.282055, 1.482919),
    0.87: (0.298589, 1.459022),
    0.88: (0.316139, 1.434162),
    0.89: (0.334823, 1.408223),
    0.90: (0.354785, 1.381059),
    0.91: (0.376205, 1.352489),
    0.92: (0.399317, 1.322280),
    0.93: (0.424428, 1.290125),
    0.94: (0.451958, 1.255602),
    0.95: (0.482512, 1.218106),
    0.96: (0.517018, 1.176710),
    0.97: (0.557031, 1.129857),
    0.98: (0.605576, 1.074522),
}


@dataclasses.dataclass
class Fields:
    """Initial macroscopic fields, float32 arrays of shape [ny, nx] (x fastest)."""
    rho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    T: np.ndarray

    def as_f64(self):
        return tuple(np.asarray(a, dtype=np.float64) for a in (self.rho, self.ux, self.uy, self.T))


def _pack(rho, ux, uy, T) -> Fields:
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Fields(f32(rho), f32(ux), f32(uy), f32(T))


def _periodic_tanh_step(x, x0, width, period, images=3):
    """sum over periodic images of tanh((x - x0 + j L)/W) - sign(j) (a smooth periodic ramp)."""
    out = np.zeros_like(x, dtype=np.float64)
    for j in range(-images, images + 1):
        out += np.tanh((x - x0 + j * period) / width)
    return out


def slab(nx, ny, t_ratio=0.90, width=4.0, noise=1e-3, seed=0, rho_v=None, rho_l=None) -> Fields:
    """Liquid slab occupying nx/4 < x <= 3nx/4 (Eq. (50) geometry) with tanh interfaces of
    width `width` grid units, plus `noise` * U[-1, 1] i.i.d. density noise.

    The profile is made exactly periodic by summing periodic images of both tanh ramps.
    """
    if rho_v is None:
        rho_v, rho_l = COEXISTENCE[round(t_ratio, 2)]
    x = np.arange(nx, dtype=np.float64)
    ramp = _periodic_tanh_step(x, nx / 4.0, width, nx) - _periodic_tanh_step(x, 3.0 * nx / 4.0, width, nx)
    prof = rho_v + 0.5 * (rho_l - rho_v) * ramp
    rho = np.broadcast_to(prof[None, :], (ny, nx)).copy()
    if noise:
        rng = np.random.default_rng(seed)
        rho += noise * rng.uniform(-1.0, 1.0, size=(ny, nx))
    T = np.full((ny, nx), t_ratio * T_CRIT)
    zero = np.zeros((ny, nx))
    return _pack(rho, zero, zero, T)


def droplet(nx, ny, radius=40.0, t_ratio=0.85, width=4.0, center=None, rho_v=None, rho_l=None) -> Fields:
    """Circular droplet (Sec. 4.2 set-up): rho = (rho_l + rho_v)/2 - (rho_l - rho_v)/2 tanh((r - R)/W),
    r the minimum-image distance to the centre, u = 0, uniform T."""
    if rho_v is None:
        rho_v, rho_l = COEXISTENCE[round(t_ratio, 2)]
    cx, cy = (nx / 2.0, ny / 2.0) if center is None else center
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    dx = np.abs(x - cx)
    dx = np.minimum(dx, nx - dx)
    dy = np.abs(y - cy)
    dy = np.minimum(dy, ny - dy)
    r = np.sqrt(dx * dx + dy * dy)
    rho = 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh((r - radius) / width)
    T = np.full((ny, nx), t_ratio * T_CRIT)
    zero = np.zeros((ny, nx))
    return _pack(rho, zero, zero, T)


def spinodal(nx, ny, t_ratio=0.80, rel_sigma=0.005, clip=2.0, seed=2, rho0=None) -> Fields:
    """Quench from the critical density: rho = rho_c (1 + rel_sigma xi), xi ~ N(0, 1) clipped
    to +-clip, i.i.d. per site; u = 0, uniform T = t_ratio T_crit."""
    rho0 = RHO_CRIT if rho0 is None else rho0
    rng = np.random.default_rng(seed)
    xi = np.clip(rng.standard_normal((ny, nx)), -clip, clip)
    rho = rho0 * (1.0 + rel_sigma * xi)
    T = np.full((ny, nx), t_ratio * T_CRIT)
    zero = np.zeros((ny, nx))
    return _pack(rho, zero, zero, T)


def smooth_random(nx, ny, seed=0, rho0=1.0, drho=0.05, u0=0.05, T0=1.0, dT=0.03, modes=3) -> Fields:
    """Smooth, band-limited random fields (a few low Fourier modes per field) with non-zero
    velocity and temperature variation: exercises every term of the force and the
    equilibrium away from rest."""
    rng = np.random.default_rng(seed)
    x = 2.0 * np.pi * np.arange(nx)[None, :] / nx
    y = 2.0 * np.pi * np.arange(ny)[:, None] / ny

    def field(amp):
        out = np.zeros((ny, nx))
        for _ in range(modes):
            kx, ky = rng.integers(-modes, modes + 1, size=2)
            ph = rng.uniform(0.0, 2.0 * np.pi)
            out += amp * rng.uniform(0.3, 1.0) * np.cos(kx * x + ky * y + ph) / modes
        return out

    return _pack(rho0 + field(drho), field(u0), field(u0), T0 + field(dT))


def uniform(nx, ny, rho=1.0, ux=0.0, uy=0.0, T=1.0) -> Fields:
    full = lambda v: np.full((ny, nx), v)
    return _pack(full(rho), full(ux), full(uy), full(T))


# Named workloads: the small parity case, the droplet, the 1024^2 throughput case.
def slab_64() -> Fields:
    """64 x 64 slab at 0.9 T_crit, tanh width 4, 1e-3 noise, seed 0."""
    return slab(64, 64, t_ratio=0.90, width=4.0, noise=1e-3, seed=0)


def droplet_256() -> Fields:
    """256 x 256 droplet of radius 40 at 0.85 T_crit, tanh width 4, u = 0."""
    return droplet(256, 256, radius=40.0, t_ratio=0.85, width=4.0)


def spinodal_1024() -> Fields:
    """1024 x 1024 quench to 0.8 T_crit from rho_c with 0.5 % Gaussian noise (clipped at 2 sigma)."""
    return spinodal(1024, 1024, t_ratio=0.80, rel_sigma=0.005, clip=2.0, seed=2)


def model_params(**overrides):
    """The paper's parameters with the a = 2, b = 0.4 fluid; keys as in the C config."""
    p = dict(PAPER_PARAMS)
    p.update(a=EOS_A, b=EOS_B)
    p.update(overrides)
    return p


def thermal_speed(T) -> float:
    return math.sqrt(float(np.max(T)))


# Batched workload: independent instances of uneven grid sizes (temperature sweep and
# droplet-radius sweep, the paper's two benchmark set-ups of Sec. 4).
BATCH_SIZES = (128, 192, 256, 384, 512)


def batch_instances(n=64, seed=3, sizes=BATCH_SIZES):
    """n instances, each drawn independently: grid N x N with N uniform over `sizes`;
    T / T_crit uniform over 0.80, 0.81, ..., 0.98 (the coexistence table); a droplet of
    radius uniform over 10..60 grid units (at most 0.35 N, so that it stays clear of its
    periodic images) or a planar slab (probability 1/2 each); tanh width 4, u = 0, no noise.
    Returns a list of (kind, N, t_ratio, radius, Fields)."""
    rng = np.random.default_rng(seed)
    temps = sorted(COEXISTENCE)
    out = []
    for _ in range(n):
        N = int(rng.choice(sizes))
        t = float(temps[int(rng.integers(len(temps)))])
        if rng.uniform() < 0.5:
            R = float(min(int(rng.integers(10, 61)), int(0.35 * N)))
            out.append(("droplet", N, t, R, droplet(N, N, radius=R, t_ratio=t, width=4.0)))
        else:
            out.append(("slab", N, t, 0.0, slab(N, N, t_ratio=t, width=4.0, noise=0.0)))
    return out


# Warm-start network: parameter shapes (per layer W[Cout, Cin, 3, 3] then b[Cout]) and
# their seeded initial values, shared by the GPU network and its tests.
CNN_CHANNELS = ((3, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 2))


def cnn_init_params(seed=0):
    """He-normal weights (the last layer scaled by 0.1, so that the initial output stays
    close to the input), zero biases; float32 flat vector."""
    rng = np.random.default_rng(seed)
    out = []
    for i, (ci, co) in enumerate(CNN_CHANNELS):
        W = rng.standard_normal((co, ci, 3, 3)) * math.sqrt(2.0 / (ci * 9))
        if i == len(CNN_CHANNELS) - 1:
            W *= 0.1
        out += [W.ravel(), np.zeros(co)]
    return np.concatenate(out).astype(np.float32)
