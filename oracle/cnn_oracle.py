"""FP64 CPU oracle of the warm-start network: a small convolutional encoder-decoder that
maps (rho0, T0, T_target) on a periodic grid to near-equilibrium (rho, T), and of the
transform that turns its prediction into the initial fields of an FFT-LB run.

TEST INFRASTRUCTURE ONLY.  This module is the plain reference the GPU network kernels are
checked against; only the test suite may import it, and it shares no code with the HIP
path.

The network is not part of the paper: it is the learned warm start whose output initialises
an FFT-LB run (the run itself stays the judge of its error).  Its definition, fixed here:

  layer  input -> output   operation (3 x 3 taps, periodic padding, cross-correlation)
  1      3  -> 32          conv, stride 1, GELU
  2      32 -> 32          conv, stride 2 (output pixel (y, x) centred on input (2y, 2x)), GELU
  3      32 -> 32          conv, stride 2, GELU
  4      32 -> 32          nearest-neighbour upsampling by 2, conv stride 1, GELU
  5      32 -> 32          upsampling by 2, conv stride 1, GELU
  6      32 -> 2           conv stride 1, linear
  output = (x_0, x_1) + layer-6 output (a correction of the normalised input density and
  temperature channels)

with conv(X)[co, y, x] = b[co] + sum_{ci, ky, kx} W[co, ci, ky, kx] X[ci, y + ky - 1, x + kx - 1]
(indices modulo the grid), GELU(z) = z Phi(z) with Phi the standard normal distribution
function, loss = mean of squared output errors, and Adam (Kingma & Ba) with bias correction.
Parameters are one flat vector: per layer W[Cout, Cin, 3, 3] then b[Cout].

bf16 rounding (round to nearest even of the FP32 value) is provided so that tests can give
both sides identical bf16 operands.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

LAYERS = ((3, 32, "s1"), (32, 32, "s2"), (32, 32, "s2"), (32, 32, "up"), (32, 32, "up"), (32, 2, "s1"))


def layer_shapes():
    return [((co, ci, 3, 3), (co,)) for ci, co, _ in LAYERS]


def num_params() -> int:
    return sum(int(np.prod(w)) + b[0] for w, b in layer_shapes())


def unpack(theta):
    """Flat parameter vector -> list of (W, b)."""
    out, o = [], 0
    for ws, bs in layer_shapes():
        n = int(np.prod(ws))
        W = theta[o:o + n].reshape(ws)
        o += n
        b = theta[o:o + bs[0]]
        o += bs[0]
        out.append((W, b))
    return out


def bf16(x):
    """Round float values to bf16 (nearest, ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def _taps():
    return [(ky, kx) for ky in range(3) for kx in range(3)]


def conv_s1(X, W, b):
    """X [N, Ci, H, Wd] -> [N, Co, H, Wd]: the definition, one tap at a time."""
    out = np.zeros((X.shape[0], W.shape[0]) + X.shape[2:])
    for ky, kx in _taps():
        # shifted[..., y, x] = X[..., y + ky - 1, x + kx - 1]
        shifted = np.roll(X, shift=(1 - ky, 1 - kx), axis=(2, 3))
        out += np.einsum("oc,nchw->nohw", W[:, :, ky, kx], shifted)
    return out + b[None, :, None, None]


def conv_s1_adjoint(G, W):
    """Adjoint of the tap sum of conv_s1 with respect to X (G: [N, Co, H, Wd])."""
    out = np.zeros((G.shape[0], W.shape[1]) + G.shape[2:])
    for ky, kx in _taps():
        t = np.einsum("oc,nohw->nchw", W[:, :, ky, kx], G)
        out += np.roll(t, shift=(ky - 1, kx - 1), axis=(2, 3))
    return out


def conv_s1_weight_grad(G, X):
    """d/dW of sum(G * conv_s1(X, W, b)), and d/db."""
    dW = np.zeros((G.shape[1], X.shape[1], 3, 3))
    for ky, kx in _taps():
        shifted = np.roll(X, shift=(1 - ky, 1 - kx), axis=(2, 3))
        dW[:, :, ky, kx] = np.einsum("nohw,nchw->oc", G, shifted)
    return dW, G.sum(axis=(0, 2, 3))


def upsample(X):
    return X.repeat(2, axis=2).repeat(2, axis=3)


def upsample_adjoint(G):
    n, c, h, w = G.shape
    return G.reshape(n, c, h // 2, 2, w // 2, 2).sum(axis=(3, 5))


def layer_forward(kind, X, W, b):
    """Pre-activation of one layer."""
    if kind == "s1":
        return conv_s1(X, W, b)
    if kind == "s2":
        return conv_s1(X, W, b)[:, :, ::2, ::2]
    return conv_s1(upsample(X), W, b)


def layer_backward(kind, X, W, G):
    """Gradients (dX, dW, db) of sum(G * layer_forward(kind, X, W, b))."""
    if kind == "s1":
        dW, db = conv_s1_weight_grad(G, X)
        return conv_s1_adjoint(G, W), dW, db
    if kind == "s2":
        Gf = np.zeros(G.shape[:2] + X.shape[2:])
        Gf[:, :, ::2, ::2] = G
        dW, db = conv_s1_weight_grad(Gf, X)
        return conv_s1_adjoint(Gf, W), dW, db
    U = upsample(X)
    dW, db = conv_s1_weight_grad(G, U)
    return upsample_adjoint(conv_s1_adjoint(G, W)), dW, db


def forward(theta, x, round_bf16=False):
    """Network output [N, 2, H, W] and the per-layer cache (inputs, pre-activations).
    round_bf16: round every layer's weights and inputs to bf16 first (what the GPU feeds
    its matrix cores), with all arithmetic in FP64."""
    params = unpack(np.asarray(theta, np.float64))
    r = bf16 if round_bf16 else (lambda a: a)
    cache = []
    h = x
    for i, ((ci, co, kind), (W, b)) in enumerate(zip(LAYERS, params)):
        Xi, Wi = r(h), r(W)
        z = layer_forward(kind, Xi, Wi, b)
        cache.append((Xi, Wi, z))
        h = gelu(z) if i < len(LAYERS) - 1 else z
    y = x[:, :2] + h
    return y, cache


def loss_and_grad(theta, x, target, round_bf16=False):
    """Mean squared error and its gradient with respect to the flat parameters."""
    y, cache = forward(theta, x, round_bf16)
    diff = y - target
    L = float(np.mean(diff * diff))
    G = 2.0 * diff / diff.size                    # dL/dy = dL/d(layer-6 output)
    grads = []
    for i in reversed(range(len(LAYERS))):
        kind = LAYERS[i][2]
        Xi, Wi, z = cache[i]
        if i < len(LAYERS) - 1:
            G = G * gelu_grad(z)
        dX, dW, db = layer_backward(kind, Xi, Wi, G)
        grads.append((dW, db))
        G = dX
    flat = []
    for dW, db in reversed(grads):
        flat += [dW.ravel(), db]
    return L, np.concatenate(flat)


def adam(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t >= 1; returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ----------------------------------------------------------------------------
# Warm-start transform: network prediction -> initial fields of the run
# ----------------------------------------------------------------------------
#
# The prediction (rho_hat / rho_c, T_hat / T_c) becomes a physical start:
#   1. the density is clipped to [1e-3 rho_c, rho_max] (rho_max < 1/b keeps the van der
#      Waals pressure of Eq. (18) finite);
#   2. one pass of the periodic binomial filter (1 2 1)/4 along x, then along y: it removes
#      the grid-scale content the upsampling layers leave (the Nyquist mode exactly), which
#      the windowed derivatives barely act on;
#   3. the total mass of the initial field is restored by moving the interfaces: the
#      deficit is added in proportion to w = |grad rho| (central differences), so the bulk
#      densities stay; a field without interfaces (sum w <= 1e-6 sum rho) is rescaled;
#      then the density is clipped again and rescaled to the exact initial mass (a closed
#      periodic system keeps its mass, and relaxes to the equilibrium that mass selects);
#   4. the temperature is uniform at the mean of the predicted temperature (equilibria are
#      isothermal), at least 1e-2 T_c.
# The run then matches the total energy of the initial state by a uniform temperature shift
# (fftlb_oracle.match_energy), since energy is the other invariant that selects the
# equilibrium.

RHO_MIN_FRACTION = 1e-3
T_MIN_FRACTION = 1e-2


def binomial_filter(g):
    """Periodic (1 2 1)/4 along x (axis 1), then along y (axis 0)."""
    g = np.asarray(g, dtype=np.float64)
    h = 0.25 * np.roll(g, 1, axis=1) + 0.5 * g + 0.25 * np.roll(g, -1, axis=1)
    return 0.25 * np.roll(h, 1, axis=0) + 0.5 * h + 0.25 * np.roll(h, -1, axis=0)


def interface_weight(rho):
    """w = |grad rho| by periodic central differences in grid units:
    0.5 sqrt((rho[x+1] - rho[x-1])^2 + (rho[y+1] - rho[y-1])^2)."""
    rho = np.asarray(rho, dtype=np.float64)
    gx = np.roll(rho, -1, axis=1) - np.roll(rho, 1, axis=1)
    gy = np.roll(rho, -1, axis=0) - np.roll(rho, 1, axis=0)
    return 0.5 * np.sqrt(gx * gx + gy * gy)


def warm_start_transform(pred, rho0, rho_c, T_c, rho_max):
    """Initial fields (rho, T) of a warm-started run from the network prediction
    pred[2, h, w] = (rho_hat / rho_c, T_hat / T_c) and the run's initial density rho0 (steps
    1-4 above; the energy match is separate).  Returns FP64 arrays (rho, T)."""
    pred = np.asarray(pred, dtype=np.float64)
    rho_min = RHO_MIN_FRACTION * rho_c
    rho = np.clip(rho_c * pred[0], rho_min, rho_max)
    rho = binomial_filter(rho)
    m0 = float(np.asarray(rho0, dtype=np.float64).sum())
    m = float(rho.sum())
    w = interface_weight(rho)
    wsum = float(w.sum())
    if wsum > 1e-6 * m:
        rho = rho + (m0 - m) * w / wsum
    else:
        rho = rho * (m0 / m)
    rho = np.clip(rho, rho_min, rho_max)
    rho = rho * (m0 / float(rho.sum()))
    t = max(float((T_c * pred[1]).mean()), T_MIN_FRACTION * T_c)
    return rho, np.full_like(rho, t)
