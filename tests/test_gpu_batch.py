"""Column plans, the autotuner and batches of instances (through the C ABI).

A plan changes only the tiling of the column passes and the radix of the column
transforms, so every plan agrees with every other to FP32 rounding of the transforms (not
bitwise: the compiler may fuse multiply-adds differently in each kernel instance, and the
radix changes the order of the butterflies).  A batch runs the same kernels as a single
solver with the same plan, so
every instance must match a single solver started from the same fields bitwise, and the
FP64 oracle to the one-step tolerance of the parity tests.
"""
import ctypes
import math
import os
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


def tensors(fld):
    return tuple(torch.from_numpy(a) for a in (fld.rho, fld.ux, fld.uy, fld.T))


def solver(fld, params=None):
    return F.Solver(*tensors(fld), params or F.Params())


def plans_for(ny, nx):
    """Every valid column plan of a grid size."""
    tw = min(16, (nx // 2) & -(nx // 2))
    cmax = min(tw, 1 << int(math.log2(max(1, min(16, 8192 // ny)))))
    mmax = min(tw, 1 << int(math.log2(max(1, min(16, 8192 // (3 * ny))))))
    out = []
    for rc in (16, 8):
        for rm in (16, 8):
            c = 1
            while c <= cmax:
                m = 1
                while m <= mmax:
                    out.append((c, m, rc, rm))
                    m *= 2
                c *= 2
    return out


@pytest.mark.parametrize("ny,nx", [(64, 64), (96, 48), (192, 96), (256, 32)])
def test_every_plan_gives_the_same_step(ny, nx):
    fld = W.smooth_random(nx, ny, seed=21, T0=1.25)
    with solver(fld) as s:
        default = s.plan
        f0 = s.get_state().clone()
        s.step(2)
        ref = s.get_state().clone()
        scale = float(ref.abs().max())
        for plan in plans_for(ny, nx):
            s.set_plan(*plan)
            assert s.plan == plan
            s.set_state(f0)
            s.step(2)
            got = s.get_state()
            if plan == default:
                assert torch.equal(got, ref), plan
            else:
                assert float((got - ref).abs().max()) < 3e-7 * scale, plan  # a few FP32 ulps of f


@pytest.mark.parametrize("ny,nx", [(64, 64), (96, 48)])
def test_every_plan_gives_the_same_diagnostics(ny, nx):
    # In the step the derivative tiles follow the convection plan; the stand-alone
    # derivative passes of the diagnostics (stage 1 again, and the residual's divergence)
    # follow multi_cols and multi_radix.  Every plan must give the same FP64 globals.
    fld = W.smooth_random(nx, ny, seed=23, T0=1.25)
    with solver(fld) as s:
        s.step(3)
        _, ref = s.moments()
        for plan in plans_for(ny, nx):
            s.set_plan(*plan)
            _, got = s.moments()
            for k in ("mass", "px", "py", "umax"):  # from the macroscopic planes: plan-independent
                assert got[k] == ref[k], (plan, k)
            # the energy's gradient term and the residual come from column transforms
            assert got["energy"] == pytest.approx(ref["energy"], rel=1e-6), plan
            assert got["residual"] == pytest.approx(ref["residual"], rel=1e-3, abs=1e-12), plan
            assert got["steps"] == ref["steps"]


def test_invalid_plans_rejected():
    fld = W.smooth_random(64, 64, seed=22)
    with solver(fld) as s:
        for bad in [(3, 1, 16, 16), (32, 1, 16, 16), (1, 0, 16, 16), (1, 1, 4, 16), (1, 1, 32, 16), (16, 32, 16, 16),
                    (1, 1, 16, 4), (1, 1, 8, 32)]:
            with pytest.raises(F.FFTLBError) as ei:
                s.set_plan(*bad)
            assert ei.value.code == F.FFTLB_EINVAL


def test_autotune_leaves_the_trajectory_unchanged(tmp_path):
    fld = W.slab(128, 64, t_ratio=0.9, width=4.0, noise=1e-3, seed=23)
    cache = str(tmp_path / "plans.txt")
    with solver(fld) as a, solver(fld) as b:
        p0 = a.plan
        a.step(5)
        best = a.autotune(reps=3, cache_path=cache)
        assert best == a.plan
        a.set_plan(*p0)
        a.step(5)
        b.step(10)
        assert torch.equal(a.get_state(), b.get_state())
        # the plan was stored and is found again without timing
        line = open(cache).read().split()
        assert line[1:3] == ["128", "64"] and tuple(int(v) for v in line[3:7]) == best
        with solver(fld) as c:
            assert c.autotune(reps=3, cache_path=cache) == best


MIXED = [(64, 64, "slab"), (96, 48, "smooth"), (48, 96, "smooth"), (128, 64, "droplet"), (64, 64, "smooth"),
         (192, 192, "droplet")]


def mixed_fields(seed=30):
    out = []
    for i, (ny, nx, kind) in enumerate(MIXED):
        if kind == "slab":
            out.append(W.slab(nx, ny, t_ratio=0.9, width=4.0, noise=1e-3, seed=seed + i))
        elif kind == "droplet":
            out.append(W.droplet(nx, ny, radius=min(nx, ny) / 5, t_ratio=0.85, width=4.0))
        else:
            out.append(W.smooth_random(nx, ny, seed=seed + i, T0=1.2))
    return out


def test_batch_instances_equal_single_solvers():
    flds = mixed_fields()
    with F.Batch([tensors(f) for f in flds]) as b:
        b.run(tol=0.0, consecutive=3, poll_every=10, max_steps=20)  # tol 0: nothing retires
        st = b.status()
        assert list(st["state"]) == [0] * len(flds)
        assert list(st["steps"]) == [20] * len(flds)
        for i, fld in enumerate(flds):
            with solver(fld) as s:
                s.step(20)
                assert torch.equal(b.instance(i).get_state(), s.get_state()), i
                _, g = s.moments()
                _, gb = b.instance(i).moments()
                assert gb["steps"] == 20 and gb["residual"] == g["residual"]
                assert abs(st["residual"][i] - g["residual"]) <= 1e-6 * g["residual"]


def test_batch_instance_matches_oracle():
    flds = mixed_fields(seed=40)
    p = F.Params()
    with F.Batch([tensors(f) for f in flds]) as b:
        b.run(tol=0.0, poll_every=3, max_steps=3)
        i = 1  # the 96 x 48 instance: a radix-3 column transform
        f0 = b.instance(i).get_state().cpu().numpy().astype(np.float64)
        b.run(tol=0.0, poll_every=1, max_steps=1)
        f1 = b.instance(i).get_state().cpu().numpy().astype(np.float64)
    ref = O.step(f0, oparams(p))
    assert np.abs(f1 - ref).max() < 3e-7 * np.abs(ref).max()


def test_batch_retires_converged_and_nonfinite_instances():
    uni = W.uniform(64, 64, rho=0.8, T=1.1)          # residual exactly 0 every step
    act = W.slab(64, 64, t_ratio=0.9, width=4.0, noise=1e-3, seed=50)
    bad = W.uniform(48, 96, rho=0.8, T=1.1)
    bad.T[7, 9] = np.nan                              # non-finite from the first step on
    with F.Batch([tensors(uni), tensors(act), tensors(bad)]) as b:
        f_uni = None
        with pytest.raises(F.FFTLBError) as ei:
            b.run(tol=1e-12, consecutive=3, poll_every=5, max_steps=40)
        assert ei.value.code == F.FFTLB_EUNSTABLE          # returned by the C ABI itself
        st = b.status()
        assert st["state"][0] == 1 and st["steps_to_tol"][0] == 5 and st["steps"][0] == 15
        assert st["state"][1] == 0 and st["steps"][1] == 40 and st["residual"][1] > 1e-12
        assert st["state"][2] == 2 and st["steps"][2] == 5
        f_uni = b.instance(0).get_state().clone()
        # the C entry point, called directly, still reports the retired non-finite instance
        rc = F.library().fftlb_batch_run(b.handle, 1e-12, 3, 5, 10,
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == F.FFTLB_EUNSTABLE
        st2 = b.status()
        assert torch.equal(b.instance(0).get_state(), f_uni)    # retired: untouched
        assert st2["steps"][0] == 15 and st2["steps"][1] == 50 and st2["steps"][2] == 5


def test_batch_autotune_applies_one_plan_per_size(tmp_path):
    flds = mixed_fields(seed=60)
    with F.Batch([tensors(f) for f in flds]) as b:
        b.autotune(reps=2, cache_path=str(tmp_path / "plans.txt"))
        plans = {}
        for i, (ny, nx, _) in enumerate(MIXED):
            plans.setdefault((ny, nx), set()).add(b.instance(i).plan)
        assert all(len(v) == 1 for v in plans.values())
        b.run(tol=0.0, poll_every=4, max_steps=8)
        for i, fld in enumerate(flds):
            with solver(fld) as s:
                s.set_plan(*b.instance(i).plan)
                s.step(8)
                assert torch.equal(b.instance(i).get_state(), s.get_state()), i


def test_batch_512_instance_matches_oracle():
    """A 512 x 512 droplet (column transforms of length 512, as in the 64-instance workload)
    beside a 96 x 48 instance: one batch step against one oracle step."""
    big = W.droplet(512, 512, radius=60, t_ratio=0.85, width=4.0)
    small = W.smooth_random(48, 96, seed=41, T0=1.2)
    p = F.Params()
    with F.Batch([tensors(big), tensors(small)]) as b:
        b.autotune(reps=2)
        b.run(tol=0.0, poll_every=2, max_steps=2)
        f0 = b.instance(0).get_state().cpu().numpy().astype(np.float64)
        b.run(tol=0.0, poll_every=1, max_steps=1)
        f1 = b.instance(0).get_state().cpu().numpy().astype(np.float64)
        plan = b.instance(0).plan
    ref = O.step(f0, oparams(p), workers=-1)
    err = np.abs(f1 - ref).max() / np.abs(ref).max()
    sys.stderr.write(f"[batch 512^2 one step, plan {plan}] max err / max f = {err:.3e}\n")
    assert err < 3e-7
