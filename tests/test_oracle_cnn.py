"""Pins of the warm-start network's CPU oracle against independent routes: torch's CPU
convolution, interpolation and automatic differentiation (float64), central finite
differences, the closed form of Adam's first steps, and torch's bf16 rounding."""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as TF

from oracle import cnn_oracle as C
from paper_1011_3582_amd import workloads as W

torch.set_default_dtype(torch.float64)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a))


def _torch_layer(kind, X, Wt, b):
    if kind == "up":
        X = TF.interpolate(X, scale_factor=2, mode="nearest")
    Xp = TF.pad(X, (1, 1, 1, 1), mode="circular")
    return TF.conv2d(Xp, Wt, b, stride=2 if kind == "s2" else 1)


@pytest.mark.parametrize("kind", ["s1", "s2", "up"])
def test_layer_matches_torch_convolution(kind):
    rng = np.random.default_rng(1)
    X = rng.standard_normal((2, 5, 8, 12))
    Wt = rng.standard_normal((4, 5, 3, 3))
    b = rng.standard_normal(4)
    ref = _torch_layer(kind, _t(X), _t(Wt), _t(b)).numpy()
    np.testing.assert_allclose(C.layer_forward(kind, X, Wt, b), ref, rtol=1e-12, atol=1e-12)


def test_gelu_is_erf_form_and_its_derivative():
    z = np.linspace(-6, 6, 1001)
    np.testing.assert_allclose(C.gelu(z), TF.gelu(_t(z), approximate="none").numpy(), rtol=1e-13, atol=1e-15)
    h = 1e-6
    fd = (C.gelu(z + h) - C.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(C.gelu_grad(z), fd, rtol=1e-7, atol=1e-9)


def _torch_net(theta, x):
    params = []
    o = 0
    for ci, co, _ in C.LAYERS:
        n = co * ci * 9
        params.append((theta[o:o + n].reshape(co, ci, 3, 3), theta[o + n:o + n + co]))
        o += n + co
    h = x
    for i, ((ci, co, kind), (Wt, b)) in enumerate(zip(C.LAYERS, params)):
        z = _torch_layer(kind, h, Wt, b)
        h = TF.gelu(z, approximate="none") if i < len(C.LAYERS) - 1 else z
    return x[:, :2] + h


def _problem(seed=2, n=2, h=8, w=8):
    rng = np.random.default_rng(seed)
    theta = W.cnn_init_params(seed).astype(np.float64)
    theta[-2:] = 0.01                       # non-zero last biases
    x = rng.uniform(0.5, 1.5, (n, 3, h, w))
    target = x[:, :2] + 0.1 * rng.standard_normal((n, 2, h, w))
    return theta, x, target


def test_forward_and_gradient_match_torch_autograd():
    theta, x, target = _problem()
    L, g = C.loss_and_grad(theta, x, target)
    th = _t(theta).requires_grad_(True)
    y = _torch_net(th, _t(x))
    Lt = ((y - _t(target)) ** 2).mean()
    Lt.backward()
    assert L == pytest.approx(float(Lt), rel=1e-12)
    np.testing.assert_allclose(g, th.grad.numpy(), rtol=1e-9, atol=1e-14)


def test_gradient_matches_finite_differences():
    theta, x, target = _problem(seed=3)
    _, g = C.loss_and_grad(theta, x, target)
    rng = np.random.default_rng(4)
    idx = np.concatenate([rng.choice(theta.size, 40, replace=False), np.arange(theta.size - 2, theta.size)])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (C.loss_and_grad(theta + e, x, target)[0] - C.loss_and_grad(theta - e, x, target)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-10), i


def test_parameter_count():
    assert C.num_params() == 3 * 32 * 9 + 32 + 4 * (32 * 32 * 9 + 32) + 32 * 2 * 9 + 2 == 38466
    assert W.cnn_init_params(0).size == C.num_params()


def test_adam_first_steps_closed_form():
    g1, g2 = np.array([0.3, -2.0, 1e-3]), np.array([0.1, 1.0, -1e-3])
    th0 = np.array([1.0, 2.0, 3.0])
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    th1, m, v = C.adam(th0, g1, np.zeros(3), np.zeros(3), 1, lr)
    np.testing.assert_allclose(th1, th0 - lr * g1 / (np.abs(g1) + eps), rtol=1e-14)
    th2, m, v = C.adam(th1, g2, m, v, 2, lr)
    mh = (b1 * (1 - b1) * g1 + (1 - b1) * g2) / (1 - b1 ** 2)
    vh = (b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2) / (1 - b2 ** 2)
    np.testing.assert_allclose(th2, th1 - lr * mh / (np.sqrt(vh) + eps), rtol=1e-13)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-8, 8, 10000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(C.bf16(x), ref)
    assert C.bf16(np.float32(1.0 + 2 ** -8)) == 1.0                  # tie to even
    assert C.bf16(np.float32(1.0 + 3 * 2 ** -8)) == 1.0 + 2 ** -6     # tie to even (up)
