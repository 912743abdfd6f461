"""The NPS scheme (filter_order 6: the nine-point stencils of Sec. 3.1 for every derivative and
for the convection term) against the FP64 oracle, which applies the stencils in real space;
the HIP path applies their Fourier symbols in column passes, splitting the packed
(DC, Nyquist) column of the row spectra by Hermitian symmetry."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import fftlb_oracle as O
from paper_1011_3582_amd import workloads as W

pytestmark = pytest.mark.gpu

F = None
NPS = 6


@pytest.fixture(autouse=True, scope="module")
def _lib():
    global F
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1011_3582_amd import fftlb as _F
    F = _F
    yield


@pytest.fixture(autouse=True)
def _announce(request):
    sys.stderr.write(f"\n[gpu-test] {request.node.nodeid}\n")
    sys.stderr.flush()
    yield


def oparams(p) -> O.Params:
    return O.Params(dx=p.dx, dy=p.dy, dt=p.dt, tau=p.tau, K=p.K, H=p.H, zeta=p.zeta, q=p.q, a=p.a, b=p.b, m=p.m,
                    conv=p.convection)


def solver(fld, p):
    return F.Solver(*(torch.from_numpy(a) for a in (fld.rho, fld.ux, fld.uy, fld.T)), p)


def state64(s):
    return s.get_state().cpu().numpy().astype(np.float64)


SHAPES = [(64, 64), (48, 96), (96, 48), (16, 2048), (2048, 16), (4, 512), (32, 8), (256, 256)]


def _fields(ny, nx, seed):
    if ny >= 16 and nx >= 16:
        return W.smooth_random(nx, ny, seed=seed, rho0=1.0, drho=0.05, u0=0.05, T0=1.2, dT=0.03)
    return W.slab(nx, ny, t_ratio=0.9, width=4.0, noise=1e-3, seed=seed)


@pytest.mark.parametrize("ny,nx", SHAPES)
def test_derivatives(ny, nx):
    """D_x, D_y and the nine-point Laplacian of a field with white noise on it (every
    wavenumber present, the x Nyquist column included) through fftlb_derivative."""
    rng = np.random.default_rng(ny * 3 + nx)
    fld = _fields(ny, nx, seed=5)
    g = (fld.rho.astype(np.float64) + 0.01 * rng.uniform(-1, 1, (ny, nx))).astype(np.float32)
    p = F.Params(m=NPS)
    D = O.Deriv(ny, nx, oparams(p))
    g64 = g.astype(np.float64)
    refs = [D.x(g64), D.y(g64), D.laplacian(g64)]
    # largest symbols: |D| <= 1/d, |Lap| <= (8 + 8/3)/d^2
    sym = np.array([1.0 / p.dx, 1.0 / p.dy, (8.0 + 8.0 / 3.0) / (p.dx * p.dy)])
    bound = 6e-8 * math.log2(nx * ny) * np.abs(g64).max() * sym
    with solver(fld, p) as s:
        for op, ref in enumerate(refs):
            got = s.derivative(torch.from_numpy(g), op).cpu().numpy()
            err = np.abs(got - ref).max()
            assert err < bound[op], (op, err, bound[op])


@pytest.mark.parametrize("ny,nx", SHAPES[:-1])
@pytest.mark.parametrize("convection", [0, 1, 4])
def test_one_step_from_shared_state(convection, ny, nx):
    """NPS + NPS (convection 0), LW + NPS (convection 1) and FL + NPS (convection 4)."""
    p = F.Params(m=NPS, convection=convection)
    with solver(_fields(ny, nx, seed=31 + convection), p) as s:
        s.step(2)
        f0 = state64(s)
        s.step(1)
        f1 = state64(s)
    ref = O.step(f0, oparams(p))
    scale = np.abs(ref).max()
    assert np.abs(f1 - ref).max() < 3e-7 * scale, np.abs(f1 - ref).max() / scale
    du, dr = f1 - f0, ref - f0
    assert np.abs(du - dr).max() < 2e-3 * np.abs(dr).max() + 1.5e-7 * scale


def test_force_and_convection_terms_match():
    """The force and the convection term of one step separately: the step from a state with the
    collision switched off (tau = inf) at dt = 1e-4, against the oracle's convection and force
    terms, each far above FP32 rounding."""
    fld = W.slab(64, 64, t_ratio=0.9, width=2.0, noise=1e-3, seed=2)
    p = F.Params(m=NPS, dt=1e-4, tau=math.inf)
    with solver(fld, p) as s:
        f0 = state64(s)
        s.step(1)
        f1 = state64(s)
    parts = O.step_parts(f0, oparams(p))
    scale = np.abs(f0).max()
    du = f1 - f0
    dr = parts.f_next - f0
    conv, force = -p.dt * parts.conv, p.dt * parts.I
    sys.stderr.write(f"[nps terms] conv {np.abs(conv).max() / scale:.2e}, force {np.abs(force).max() / scale:.2e}, "
                     f"err {np.abs(du - dr).max() / scale:.2e}\n")
    assert np.abs(conv).max() > 1e-4 * scale and np.abs(force).max() > 1e-5 * scale
    assert np.abs(du - dr).max() < 2e-3 * np.abs(dr).max() + 1.5e-7 * scale


def test_slab64_100_steps():
    fld = W.slab_64()
    p = F.Params(m=NPS)
    with solver(fld, p) as s:
        s.step(100)
        f = state64(s)
        _, g = s.moments()
    ref = O.run(O.feq(*fld.as_f64()), oparams(p), 100)
    rho, ux, uy, T = O.moments(f)
    orho, oux, ouy, oT = O.moments(ref)
    vt = math.sqrt(oT.max())
    errs = dict(f=float(np.abs(f - ref).max() / np.abs(ref).max()),
                rho=float(np.abs(rho - orho).max() / np.abs(orho).max()),
                T=float(np.abs(T - oT).max() / np.abs(oT).max()),
                u=float(max(np.abs(ux - oux).max(), np.abs(uy - ouy).max()) / vt))
    sys.stderr.write(f"[slab64 NPS, 100 steps] {errs}\n")
    for k, v in errs.items():
        assert v < 1e-5, (k, v)
    mass0 = float(fld.rho.astype(np.float64).sum() * p.dx * p.dy)
    assert abs(g["mass"] - mass0) < 1e-6 * mass0
    # the global energy uses the NPS gradient of rho
    assert g["energy"] == pytest.approx(O.globals_of(ref, oparams(p))["energy"], rel=1e-5)


def test_rejected_on_a_rectangular_lattice():
    fld = _fields(64, 64, seed=1)
    with pytest.raises(F.FFTLBError):
        solver(fld, F.Params(m=NPS, dy=1.0 / 200.0))


def test_batch_with_nps_and_windowed_instances_is_bitwise_solo():
    flds = [W.smooth_random(64, 64, seed=50 + k, T0=1.2) for k in range(3)]
    params = [F.Params(m=NPS), F.Params(), F.Params(m=NPS, convection=3)]
    b = F.Batch([tuple(torch.from_numpy(a) for a in (f.rho, f.ux, f.uy, f.T)) for f in flds], params=params)
    try:
        b.run(tol=0.0, consecutive=3, poll_every=10, max_steps=30)
        got = [b.instance(i).get_state().cpu().numpy() for i in range(3)]
    finally:
        b.close()
    for fld, p, g in zip(flds, params, got):
        with solver(fld, p) as s:
            s.step(30)
            assert np.array_equal(s.get_state().cpu().numpy(), g)
