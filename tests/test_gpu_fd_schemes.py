"""The finite-difference convection schemes of Sec. 3.1 (fftlb_config.convection: LW, MLW1,
MLW2, FL, with the central difference for the force, filter_order 5) against the FP64 oracle,
which applies them as the printed stencils in real space; the HIP path applies LW, MLW1 and
MLW2 as their Fourier symbols in a column pass over all 32 moving populations, and the flux
limiter (nonlinear) in a real-space kernel along each population's characteristic line."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import fftlb_oracle as O
from paper_1011_3582_amd import workloads as W

pytestmark = pytest.mark.gpu

F = None
SCHEMES = (1, 2, 3, 4)   # LW, MLW1, MLW2, FL


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


# square, 3 * 2^p, 2048-point rows and columns, 4-point columns, rows of 8
SHAPES = [(64, 64), (48, 96), (16, 2048), (2048, 16), (4, 512), (32, 8)]


def _fields(ny, nx, seed):
    if ny >= 16 and nx >= 16:
        return W.smooth_random(nx, ny, seed=seed, rho0=1.0, drho=0.05, u0=0.05, T0=1.2, dT=0.03)
    return W.slab(nx, ny, t_ratio=0.9, width=4.0, noise=1e-3, seed=seed)


@pytest.mark.parametrize("ny,nx", SHAPES)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_one_step_from_shared_state(scheme, ny, nx):
    p = F.Params(m=5, convection=scheme)
    with solver(_fields(ny, nx, seed=21 + scheme), p) as s:
        s.step(2)
        f0 = state64(s)
        s.step(1)
        f1 = state64(s)
    ref = O.step(f0, oparams(p))
    scale = np.abs(ref).max()
    assert np.abs(f1 - ref).max() < 3e-7 * scale, np.abs(f1 - ref).max() / scale
    du, dr = f1 - f0, ref - f0
    assert np.abs(du - dr).max() < 2e-3 * np.abs(dr).max() + 1.5e-7 * scale


def test_each_scheme_term_matches():
    """The differences LW - CD, MLW1 - LW (the R3 term), MLW2 - MLW1 (the R4 term) and FL - CD of
    one step from the same state: a sharp slab and dt = 4e-4 (CFL numbers up to 0.44), where each
    term is 1e-4..1e-3 of the state, far above FP32 rounding."""
    fld = W.slab(64, 64, t_ratio=0.9, width=2.0, noise=1e-3, seed=2)
    out, ref = {}, {}
    f0 = None
    for conv in (0, 1, 2, 3, 4):
        p = F.Params(m=5, dt=4e-4, convection=conv)
        with solver(fld, p) as s:
            g0 = state64(s)
            if f0 is None:
                f0 = g0
            s.set_state(torch.from_numpy(f0.astype(np.float32)))
            s.step(1)
            out[conv] = state64(s)
        ref[conv] = O.step(f0, oparams(p))
    scale = np.abs(ref[0]).max()
    for a, b, name in ((1, 0, "LW - CD"), (2, 1, "R3"), (3, 2, "R4"), (4, 0, "FL - CD")):
        dg, do = out[a] - out[b], ref[a] - ref[b]
        err = np.abs(dg - do).max()
        sys.stderr.write(f"[{name}] max {np.abs(do).max() / scale:.2e}, err {err / scale:.2e} of the state\n")
        assert np.abs(do).max() > 1e-4 * scale
        assert err < 2e-3 * np.abs(do).max() + 3e-7 * scale, (name, err / np.abs(do).max())


@pytest.mark.parametrize("scheme", SCHEMES)
def test_slab64_100_steps(scheme):
    fld = W.slab_64()
    p = F.Params(m=5, convection=scheme)
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
    sys.stderr.write(f"[slab64 scheme {scheme}, 100 steps] {errs}\n")
    for k, v in errs.items():
        assert v < 1e-5, (k, v)
    # the stencils conserve mass
    mass0 = float(fld.rho.astype(np.float64).sum() * p.dx * p.dy)
    assert abs(g["mass"] - mass0) < 1e-6 * mass0


def test_batch_of_mixed_schemes_is_bitwise_solo():
    """Instances of one grid size with different convection schemes share a batch (grouped by
    scheme): each evolves bitwise as it does alone."""
    flds = [W.smooth_random(64, 64, seed=40 + k, T0=1.2) for k in range(4)]
    schemes = [0, 1, 3, 4]
    params = [F.Params(m=5, convection=c) for c in schemes]
    b = F.Batch([tuple(torch.from_numpy(a) for a in (f.rho, f.ux, f.uy, f.T)) for f in flds], params=params)
    try:
        b.run(tol=0.0, consecutive=3, poll_every=10, max_steps=30)
        got = [b.instance(i).get_state().cpu().numpy() for i in range(4)]
    finally:
        b.close()
    for fld, p, g in zip(flds, params, got):
        with solver(fld, p) as s:
            s.step(30)
            assert np.array_equal(s.get_state().cpu().numpy(), g)


@pytest.mark.parametrize("m,scheme", [(5, 1), (5, 4), (6, 0)])
def test_compensated_state_with_schemes(m, scheme):
    """The comparison schemes with the compensated state (precision 1; the collide variant that
    takes every convection spectrum from a pass and keeps the low parts): one step from a shared
    state against the oracle, and 20 steps against the FP32 run of the same scheme."""
    fld = _fields(64, 64, seed=60 + scheme)
    p = F.Params(m=m, convection=scheme, precision=1)
    with solver(fld, p) as s:
        s.step(2)
        f0 = state64(s)
        s.step(1)
        f1 = state64(s)
        s.step(17)
        f20 = state64(s)
    ref = O.step(f0, oparams(p))
    scale = np.abs(ref).max()
    assert np.abs(f1 - ref).max() < 3e-7 * scale, np.abs(f1 - ref).max() / scale
    p32 = F.Params(m=m, convection=scheme)
    with solver(fld, p32) as s:
        s.step(20)
        g20 = state64(s)
    assert np.abs(f20 - g20).max() < 2e-6 * scale


def test_batch_of_many_flux_limiter_instances_is_bitwise_solo():
    """Nine flux-limiter instances in one batch (two launches of the stencil and the row transforms
    per step, eight instances in the first): each evolves bitwise as it does alone."""
    flds = [W.smooth_random(64, 64, seed=70 + k, T0=1.2) for k in range(9)]
    p = F.Params(m=5, convection=4)
    b = F.Batch([tuple(torch.from_numpy(a) for a in (f.rho, f.ux, f.uy, f.T)) for f in flds], params=p)
    try:
        b.run(tol=0.0, consecutive=3, poll_every=10, max_steps=20)
        got = [b.instance(i).get_state().cpu().numpy() for i in range(9)]
    finally:
        b.close()
    for k in (0, 7, 8):
        with solver(flds[k], p) as s:
            s.step(20)
            assert np.array_equal(s.get_state().cpu().numpy(), got[k])
