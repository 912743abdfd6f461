"""What the trained warm-start network gains over the plain method, on a small problem.

Relaxed fields are produced by the solver itself (batched FFT-LB runs of 64 x 64 slabs and
droplets at 0.80..0.98 T_c until the residual dt max|D.(rho u)| stays below 1e-6), the
network is trained on them on the GPU, and held-out instances are run to the same residual
tolerance from their initial fields (cold) and from the network's prediction (warm).
"""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    sys.stderr.write(f"\n[gpu-test] {request.node.nodeid}\n")
    sys.stderr.flush()
    yield


def test_trained_network_shortens_relaxation():
    from paper_1011_3582_amd import warmstart as WS
    from paper_1011_3582_amd import workloads as W
    size, tol = 64, 1e-6
    x, y, steps = WS.make_dataset(48, 500, size, tol, 20000, per_batch=48)
    net, hist, _ = WS.train(x, y, epochs=60, batch=8, lr=2e-3)
    assert hist[-1] < 0.2 * hist[0]
    # the prediction is closer to the relaxed field than the initial field is
    xe, ye, _ = WS.make_dataset(8, 900, size, tol, 20000, per_batch=8)
    pred = net.forward(torch.from_numpy(xe)).cpu().numpy()
    err_pred = np.sqrt(np.mean((pred[:, 0] - ye[:, 0]) ** 2))
    err_init = np.sqrt(np.mean((xe[:, 0] - ye[:, 0]) ** 2))
    assert err_pred < 0.5 * err_init, (err_pred, err_init)
    # held-out runs to the same tolerance: fewer steps from the warm start
    ev = WS.evaluate(net, 8, 900, size, tol, 20000)
    sys.stderr.write(f"[gpu-test] cold {ev['steps_cold']} warm {ev['steps_warm']}\n")
    # capped runs count as the cap in the medians
    assert ev["warm_capped"] <= ev["cold_capped"], ev
    assert ev["steps_warm_median"] < ev["steps_cold_median"], ev
    net.close()
