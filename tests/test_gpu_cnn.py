"""The warm-start network's HIP kernels (bf16 matrix cores, FP32 accumulation) against the
FP64 CPU oracle.

Layer by layer, both sides get identical bf16 operands (the GPU's own FP32 activations and
parameters, rounded to bf16 by the oracle exactly as the GPU rounds them on the way into
the matrix cores), so the only difference left is FP32 accumulation of at most 1152
products: |GPU - oracle| <= 2e-5 of the largest magnitude.  End to end, the GPU also rounds
the backward-pass gradients to bf16, which the plain oracle does not: there the gradient
agrees to about 1e-2 in norm.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import cnn_oracle as C
from paper_1011_3582_amd import workloads as W

pytestmark = pytest.mark.gpu

N = None


@pytest.fixture(autouse=True, scope="module")
def _lib():
    global N
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1011_3582_amd import cnn as _N
    N = _N
    yield


@pytest.fixture(autouse=True)
def _announce(request):
    sys.stderr.write(f"\n[gpu-test] {request.node.nodeid}\n")
    sys.stderr.flush()
    yield


def _shapes(h, w):
    out, H, Wd = [], h, w
    for ci, co, kind in C.LAYERS:
        if kind == "s2":
            H, Wd = H // 2, Wd // 2
        elif kind == "up":
            H, Wd = H * 2, Wd * 2
        out.append((co, H, Wd))
    return out


def _problem(h=32, w=32, n=2, seed=7):
    rng = np.random.default_rng(seed)
    theta = W.cnn_init_params(seed).astype(np.float64)
    theta[-2:] = 0.02
    x = rng.uniform(0.3, 1.6, (n, 3, h, w)).astype(np.float32)
    target = (x[:, :2] + 0.05 * rng.standard_normal((n, 2, h, w))).astype(np.float32)
    return theta.astype(np.float32), x, target


def _close(got, ref, rel):
    scale = max(float(np.abs(ref).max()), 1e-30)
    err = float(np.abs(np.asarray(got, np.float64) - ref).max())
    assert err <= rel * scale, (err, scale)


def test_forward_layer_by_layer():
    h = w = 32
    theta, x, _ = _problem(h, w)
    net = N.Network(h, w, 2, torch.from_numpy(theta))
    y = net.forward(torch.from_numpy(x)).cpu().numpy()
    params = C.unpack(theta.astype(np.float64))
    inp = x.astype(np.float64)
    for l, ((ci, co, kind), (Wl, bl), shp) in enumerate(zip(C.LAYERS, params, _shapes(h, w))):
        z = net.buffer(l + 1, 0, 2, shp).cpu().numpy()
        ref = C.layer_forward(kind, C.bf16(inp), C.bf16(Wl), bl)
        _close(z, ref, 2e-5)
        if l < len(C.LAYERS) - 1:
            a = net.buffer(l + 1, 2, 2, shp).cpu().numpy()
            _close(a, C.gelu(z.astype(np.float64)), 1e-6)
            inp = a.astype(np.float64)
    _close(y, x[:, :2].astype(np.float64) + z.astype(np.float64), 1e-7)
    net.close()


def test_backward_layer_by_layer():
    h = w = 32
    theta, x, target = _problem(h, w, seed=8)
    net = N.Network(h, w, 2, torch.from_numpy(theta))
    L, g = net.gradient(torch.from_numpy(x), torch.from_numpy(target))
    g = g.cpu().numpy().astype(np.float64)
    shp = _shapes(h, w)
    y = net.buffer(6, 2, 2, shp[-1]).cpu().numpy().astype(np.float64)
    d = y - target
    assert float(L.item()) == pytest.approx(float(np.mean(d * d)), rel=1e-6)
    params = C.unpack(theta.astype(np.float64))
    offs = np.cumsum([0] + [Wl.size + bl.size for Wl, bl in params])
    for l in reversed(range(len(C.LAYERS))):
        kind = C.LAYERS[l][2]
        Wl, bl = params[l]
        dz = net.buffer(l + 1, 1, 2, shp[l]).cpu().numpy().astype(np.float64)
        if l == len(C.LAYERS) - 1:
            _close(dz, 2.0 * d / d.size, 1e-6)
        X = x.astype(np.float64) if l == 0 else net.buffer(l, 2, 2, shp[l - 1]).cpu().numpy().astype(np.float64)
        dX, dW, db = C.layer_backward(kind, C.bf16(X), C.bf16(Wl), C.bf16(dz))
        gl = g[offs[l]:offs[l + 1]]
        _close(gl[:Wl.size], dW.ravel(), 2e-5)
        # the bias gradient sums bf16-rounded dZ values
        _close(gl[Wl.size:], db, 2e-5)
        if l > 0:
            zprev = net.buffer(l, 0, 2, shp[l - 1]).cpu().numpy().astype(np.float64)
            dzprev = net.buffer(l, 1, 2, shp[l - 1]).cpu().numpy()
            _close(dzprev, dX * C.gelu_grad(zprev), 2e-5)
    net.close()


def test_gradient_end_to_end_against_fp64():
    h = w = 32
    theta, x, target = _problem(h, w, seed=9)
    net = N.Network(h, w, 2, torch.from_numpy(theta))
    L, g = net.gradient(torch.from_numpy(x), torch.from_numpy(target))
    g = g.cpu().numpy().astype(np.float64)
    L_ref, g_ref = C.loss_and_grad(theta.astype(np.float64), x.astype(np.float64), target.astype(np.float64))
    assert float(L.item()) == pytest.approx(L_ref, rel=2e-2)
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    cos = float(g @ g_ref / (np.linalg.norm(g) * np.linalg.norm(g_ref)))
    assert rel < 2e-2 and cos > 0.9995, (rel, cos)
    net.close()


def test_adam_step_matches_oracle():
    h = w = 16
    theta, x, target = _problem(h, w, n=1, seed=10)
    net = N.Network(h, w, 1, torch.from_numpy(theta))
    _, g = net.gradient(torch.from_numpy(x[:1]), torch.from_numpy(target[:1]))
    g = g.cpu().numpy().astype(np.float64)
    from paper_1011_3582_amd import fftlb as F
    F._check(N.library().fftlb_cnn_adam_step(net.handle, 1e-3, N._stream(net.device)), "adam")
    got = net.params.cpu().numpy().astype(np.float64)
    ref, _, _ = C.adam(theta.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, 1e-3)
    np.testing.assert_allclose(got, ref, rtol=0, atol=2e-7 * np.abs(ref).max())
    net.close()


def test_training_reduces_the_loss():
    h = w = 32
    rng = np.random.default_rng(11)
    theta = W.cnn_init_params(11)
    x = rng.uniform(0.5, 1.5, (4, 3, h, w)).astype(np.float32)
    # a smooth target the network can learn: a periodic 3-point average of the input channels
    t = x[:, :2].copy()
    t = (np.roll(t, 1, 2) + t + np.roll(t, -1, 2)) / 3.0
    net = N.Network(h, w, 4, torch.from_numpy(theta))
    xs, ts = torch.from_numpy(x), torch.from_numpy(t.astype(np.float32))
    first = float(net.train_step(xs, ts, 2e-3).item())
    for _ in range(300):
        last = float(net.train_step(xs, ts, 2e-3).item())
    assert last < 0.7 * first, (first, last)
    # the weight gradient is summed in a fixed order: a second run is bitwise the same
    net2 = N.Network(h, w, 4, torch.from_numpy(theta))
    for _ in range(301):
        net2.train_step(xs, ts, 2e-3)
    assert torch.equal(net.params, net2.params)
    net.close()
    net2.close()


def test_gradient_is_deterministic():
    h = w = 64
    theta, x, target = _problem(h, w, n=2, seed=13)
    net = N.Network(h, w, 2, torch.from_numpy(theta))
    l1, g1 = net.gradient(torch.from_numpy(x), torch.from_numpy(target))
    g1, l1 = g1.clone(), float(l1)
    l2, g2 = net.gradient(torch.from_numpy(x), torch.from_numpy(target))
    assert torch.equal(g1, g2) and l1 == float(l2)
    net.close()


def _prediction(n, seed, deficit):
    """A seeded synthetic prediction of a droplet run: a sharper, smaller droplet than the
    initial field (so mass is missing), noise, and a few values beyond both clip bounds."""
    rng = np.random.default_rng(seed)
    fld = W.droplet(n, n, radius=n / 5, t_ratio=0.85, width=4.0)
    pr = W.droplet(n, n, radius=n / 5 * (1 - deficit), t_ratio=0.85, width=1.5).rho.astype(np.float64)
    pr *= 1 + 0.01 * rng.standard_normal((n, n))
    pr[3, 5], pr[n // 2, n // 3], pr[n - 2, 7] = 9.0, -1.0, 0.0
    pt = 0.85 + 0.01 * rng.standard_normal((n, n))
    pred = np.stack([pr / W.RHO_CRIT, pt]).astype(np.float32)
    return fld, pred


@pytest.mark.parametrize("n", [64, 256])
def test_warm_start_transform_matches_oracle(n):
    """fftlb_cnn_project against the FP64 oracle's warm_start_transform, element by element,
    from the same FP32 prediction.  The GPU chain (product, two filter sums, shift, clip,
    rescale) rounds each value about eight times in FP32 (<= 5e-7 relative); the shift
    coefficient (M0 - M)/sum w carries the FP32 rounding of M (~1e-7 M), amplified by
    M / sum w (~1e2 for these droplets) into at most ~3e-6 of rho at the interfaces."""
    fld, pred = _prediction(n, seed=n + 1, deficit=0.1)
    rho_max = 0.95 / W.EOS_B
    net = N.Network(n, n, 1, torch.from_numpy(W.cnn_init_params(0)))
    rho, T = net.project(torch.from_numpy(pred), torch.from_numpy(fld.rho), W.RHO_CRIT, W.T_CRIT, rho_max)
    rho, T = rho.cpu().numpy().astype(np.float64), T.cpu().numpy().astype(np.float64)
    net.close()
    ref_rho, ref_T = C.warm_start_transform(pred.astype(np.float64), fld.rho.astype(np.float64), W.RHO_CRIT,
                                            W.T_CRIT, rho_max)
    err = np.abs(rho - ref_rho).max() / np.abs(ref_rho).max()
    sys.stderr.write(f"[warm-start transform {n}^2] max rel err rho {err:.2e}\n")
    assert err < 5e-6
    assert np.abs(T - ref_T).max() < 1e-6 * ref_T.max()
    assert rho.sum() == pytest.approx(fld.rho.astype(np.float64).sum(), rel=1e-6)
    # the shift moved the interfaces: the prediction's own mass was ~10 % short
    assert abs(C.binomial_filter(np.clip(W.RHO_CRIT * pred[0].astype(np.float64), 0, rho_max)).sum()
               - fld.rho.sum()) > 0.03 * fld.rho.sum()


def test_match_energy_matches_oracle():
    from oracle import fftlb_oracle as O
    from paper_1011_3582_amd import fftlb as F
    n = 128
    fld = W.droplet(n, n, radius=20, t_ratio=0.85, width=4.0)
    p = F.Params()
    op = O.Params(dx=p.dx, dy=p.dy, dt=p.dt, tau=p.tau, K=p.K, H=p.H, zeta=p.zeta, q=p.q, a=p.a, b=p.b, m=p.m)
    T_pred = np.full_like(fld.T, 0.87 * W.T_CRIT)
    with F.Solver(torch.from_numpy(fld.rho), torch.from_numpy(fld.ux), torch.from_numpy(fld.uy),
                  torch.from_numpy(fld.T), p) as cold, \
            F.Solver(torch.from_numpy(fld.rho), torch.from_numpy(fld.ux), torch.from_numpy(fld.uy),
                     torch.from_numpy(T_pred), p) as warm:
        E0 = cold.poll()["energy"]
        f = warm.get_state().cpu().numpy().astype(np.float64)
        warm.match_energy(E0)
        (rho, ux, uy, T), g = warm.moments()
        T = T.cpu().numpy().astype(np.float64)
    r, u, v, t = O.moments(f)                        # the FP32 state the GPU shifted
    ref = O.match_energy(r, u, v, t, E0, op)
    # T as the moments of the restarted FP32 state give it back (~1e-6 relative, Eq. (9))
    assert np.abs(T - ref).max() < 1e-6 * ref.max()
    assert abs(ref.mean() - 0.87 * W.T_CRIT) > 1e-3     # the shift is not trivial
    # the restarted state carries the initial energy (its FP64 sum over FP32 fields)
    scale = float((np.abs(r * t) + p.a * r * r).sum() * p.dx * p.dy)
    assert abs(g["energy"] - E0) < 1e-6 * scale


def test_warm_start_keeps_the_mass():
    h = w = 64
    fld = W.droplet(w, h, radius=12, t_ratio=0.85, width=4.0)
    net = N.Network(h, w, 1, torch.from_numpy(W.cnn_init_params(12)))
    rho, T = net.warm_start(torch.from_numpy(fld.rho), torch.from_numpy(fld.T), float(fld.T[0, 0]),
                            W.RHO_CRIT, W.T_CRIT, 0.95 / W.EOS_B)
    rho, T = rho.cpu().numpy(), T.cpu().numpy()
    assert rho.sum(dtype=np.float64) == pytest.approx(fld.rho.sum(dtype=np.float64), rel=2e-7)
    assert (rho > 0).all() and (T > 0).all() and rho.max() <= 0.95 / W.EOS_B * 1.01
    assert np.ptp(T) == 0.0                           # uniform temperature
    net.close()
