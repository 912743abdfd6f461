"""fftlb_derivative_static, the allocation-free variant of fftlb_derivative (its spectral
planes and tables in a static device array), against fftlb_derivative on a solver handle.

Both run the same three kernels (forward row transforms, the derivative column pass, inverse
row transforms); the static variant computes its twiddle and windowed-wavenumber tables on
the device (FP64, rounded to FP32) where fftlb_init computes them on the host, so the two
agree to FP32 rounding of the transforms: |D g - D' g| <= eps log2(nx ny) max|g| k_max
(eps = 6e-8; k_max^2 for the Laplacian), the bound of the derivative parity tests.  Two calls
in a row, the second on a smaller grid (the array keeps the first call's contents)."""
import ctypes
import math
import sys

import numpy as np
import pytest
import torch

from oracle import fftlb_oracle as O
from paper_1011_3582_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    sys.stderr.write(f"\n[gpu-test] {request.node.nodeid}\n")
    sys.stderr.flush()
    yield


def test_static_derivative_matches_the_handle_path_twice():
    from paper_1011_3582_amd import fftlb as F
    lib = F.library()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for ny, nx, seed in [(256, 512, 1), (64, 32, 2)]:
        rng = np.random.default_rng(seed)
        fld = W.smooth_random(nx, ny, seed=seed, T0=1.2)
        g = (fld.rho.astype(np.float64) + 0.01 * rng.uniform(-1, 1, (ny, nx))).astype(np.float32)
        p = F.Params(m=4, dy=1 / 200)
        cfg = p.config(nx, ny)
        gt = torch.from_numpy(g).cuda()
        kx = np.abs(O.kappa(nx, p.dx, p.m)).max()
        ky = np.abs(O.kappa(ny, p.dy, p.m)).max()
        kmax = [kx, ky, kx * kx + ky * ky]
        with F.Solver(*(torch.from_numpy(a) for a in (fld.rho, fld.ux, fld.uy, fld.T)), p) as s:
            for op in range(3):
                ref = s.derivative(gt, op)
                out = torch.full_like(gt, float("nan"))
                rc = lib.fftlb_derivative_static(ctypes.byref(cfg), ctypes.c_void_p(gt.data_ptr()),
                                                 ctypes.c_void_p(out.data_ptr()), op, stream)
                assert rc == F.FFTLB_OK, lib.fftlb_last_error().decode()
                err = float((out - ref).abs().max())
                bound = 6e-8 * math.log2(nx * ny) * float(np.abs(g).max()) * kmax[op]
                sys.stderr.write(f"[static derivative {ny}x{nx} op {op}] max diff {err:.2e} (bound {bound:.2e})\n")
                assert err <= bound, (ny, nx, op, err, bound)
