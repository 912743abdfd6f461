"""The compensated state (fftlb_config.precision = 1: f = hi + lo, both FP32) against the FP64
oracle, and against the plain FP32 state where increments fall below half an ulp.

An FP32 state rounds f + increment once per step, so an increment smaller than half an ulp
of f (about 3e-8 f) is lost: near equilibrium such a state stops evolving at a floor.  The
compensated update keeps the rounding error in lo, so the same increments accumulate."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import fftlb_oracle as O
from paper_1011_3582_amd import workloads as W

pytestmark = pytest.mark.gpu

F = None


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
    return O.Params(dx=p.dx, dy=p.dy, dt=p.dt, tau=p.tau, K=p.K, H=p.H, zeta=p.zeta, q=p.q, a=p.a, b=p.b, m=p.m)


def solver(fld, p):
    return F.Solver(*(torch.from_numpy(a) for a in (fld.rho, fld.ux, fld.uy, fld.T)), p)


def state64(s):
    return s.get_state().cpu().numpy().astype(np.float64)


def test_workspace_grows_by_the_low_parts():
    a = F.workspace_bytes(64, 64, F.Params())
    b = F.workspace_bytes(64, 64, F.Params(precision=1))
    assert b - a >= 33 * 64 * 64 * 4


@pytest.mark.parametrize("case", ["smooth64", "droplet_96x48"])
def test_compensated_step_matches_oracle(case):
    fld = W.smooth_random(64, 64, seed=31, T0=1.2) if case == "smooth64" else \
        W.droplet(48, 96, radius=12, t_ratio=0.85, width=3.0)
    p = F.Params(precision=1)
    with solver(fld, p) as s:
        s.step(3)
        f0 = state64(s)          # hi; lo (below half an ulp) is part of the one-step tolerance
        s.step(1)
        f1 = state64(s)
    ref = O.step(f0, oparams(p))
    scale = np.abs(ref).max()
    assert np.abs(f1 - ref).max() < 3e-7 * scale


def test_compensated_slab64_100_steps_within_target():
    fld = W.slab_64()
    errs = {}
    for prec in (0, 1):
        p = F.Params(precision=prec)
        with solver(fld, p) as s:
            s.step(100)
            f = state64(s)
        ref = O.run(O.feq(*fld.as_f64()), oparams(p), 100)
        errs[prec] = float(np.abs(f - ref).max() / np.abs(ref).max())
    sys.stderr.write(f"[slab64 100 steps] max rel err f: FP32 {errs[0]:.2e}, compensated {errs[1]:.2e}\n")
    assert errs[1] < 1e-5 and errs[1] <= 1.5 * errs[0]


def test_increments_below_half_an_ulp_accumulate():
    """A uniform state plus a non-equilibrium mode that carries no mass, momentum or energy
    (+e on the +-x populations of speed group 1, -e on its +-y populations): without
    gradients the step is plain BGK relaxation, so the mode decays as (1 - dt/tau)^n
    exactly (oracle).  With e = 1e-5 f the per-step decrement dt/tau e = 1e-8 f is below
    half an FP32 ulp of f: the FP32 state keeps the mode, the compensated state follows the
    decay."""
    ny, nx = 16, 32
    p0 = F.Params()
    fld = W.uniform(nx, ny, rho=1.0, T=1.0)
    f0 = O.feq(*fld.as_f64())
    eps = 1e-5 * f0[1]
    f0[1] += eps
    f0[5] += eps
    f0[3] -= eps
    f0[7] -= eps
    f0 = f0.astype(np.float32)
    n = 700
    f064 = f0.astype(np.float64)
    amp0 = float(f064[1, 0, 0] - O.feq(*O.moments(f064))[1, 0, 0])   # the mode of the FP32 state
    ref = O.run(f064, oparams(p0), n)
    ref_amp = ref[1, 0, 0] - O.feq(*O.moments(ref))[1, 0, 0]
    assert ref_amp == pytest.approx(amp0 * (1 - p0.dt / p0.tau) ** n, rel=1e-6)   # the oracle's BGK decay
    amps = {}
    for prec in (0, 1):
        with solver(fld, F.Params(precision=prec)) as s:
            s.set_state(torch.from_numpy(f0))
            s.step(n)
            f = state64(s)
        amps[prec] = float(np.median(f[1] - O.feq(*O.moments(f))[1]))
    sys.stderr.write(f"[sub-ulp mode] initial {amp0:.3e}, FP32 {amps[0]:.3e}, compensated {amps[1]:.3e}, "
                     f"oracle {ref_amp:.3e}\n")
    ulp = np.spacing(np.float32(f0[1, 0, 0]))
    assert abs(amps[0] - amp0) < ulp                 # FP32: the mode does not decay at all
    assert abs(amps[1] - ref_amp) < 2 * ulp           # compensated: as the oracle (to hi's rounding)
    assert ref_amp < 0.6 * amp0


def test_batch_mixes_precisions_bitwise():
    a = W.slab(64, 64, t_ratio=0.9, width=4.0, noise=1e-3, seed=33)
    b = W.droplet(48, 96, radius=12, t_ratio=0.85, width=3.0)
    params = [F.Params(precision=1), F.Params(precision=0), F.Params(precision=1)]
    flds = [a, a, b]
    with F.Batch([tuple(torch.from_numpy(x) for x in (f.rho, f.ux, f.uy, f.T)) for f in flds], params) as bt:
        bt.run(tol=0.0, poll_every=10, max_steps=30)
        for i, (f, p) in enumerate(zip(flds, params)):
            with solver(f, p) as s:
                s.step(30)
                assert torch.equal(bt.instance(i).get_state(), s.get_state()), i
        # the two precisions of the same slab differ (by the accumulated sub-ulp increments)
        assert not torch.equal(bt.instance(0).get_state(), bt.instance(1).get_state())
