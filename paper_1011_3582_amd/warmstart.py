"""Learned warm start of FFT-LB runs: data from the solver, training and evaluation.

1. relax(): run batches of instances (droplets and slabs at 0.80..0.98 T_c on N x N grids)
   with the batched solver until their residual stays below a tolerance; the relaxed
   (rho, T) fields are the training targets, (rho0 / rho_c, T0 / T_c, T / T_c) the inputs.
2. train(): Adam on the mean squared error, through the library's bf16 matrix-core
   kernels (forward, backward and update all run on the GPU).
3. evaluate(): held-out instances started cold (from their initial fields) and warm (from
   f^eq of the network's prediction, with the mass and the total energy of the cold start)
   in one batch, each run until its
   residual stays below the evaluation tolerance; steps to tolerance compared.  Also the
   best-of-two start: both starts run a short probe, the one with the smaller residual
   continues (its cost counts the other start's probe steps too).

Run as `python -m paper_1011_3582_amd.warmstart` for the full experiment; it prints one
JSON line.  Everything here orchestrates calls into the HIP library.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import cnn as N
from . import fftlb as F
from . import workloads as W


def log(msg):
    print(f"[warmstart] {msg}", file=sys.stderr, flush=True)


def _tensors(fl):
    return tuple(torch.from_numpy(np.ascontiguousarray(a)) for a in fl)


def run_batch(fields, tol, cap, chunk=20000, poll=100, probe=0, energy_from=None, trace=False, precision=0):
    """Run instances (list of (rho, ux, uy, T) arrays) until each has retired or `cap` steps.
    Returns (status dict, [(rho, T) numpy of every instance], wall seconds); with probe > 0
    the status also holds "probe_residual", every instance's residual after `probe` steps.
    energy_from {i: j}: before the run, instance i takes the total energy of instance j's
    initial state (fftlb_match_energy).  trace: the status also holds "trace", the steps and
    every instance's residual after each chunk.  precision: the state of every instance
    (0: FP32, 1: compensated, for tolerances below the FP32 floor)."""
    b = F.Batch([_tensors(f) for f in fields], params=F.Params(precision=precision))
    for i, j in (energy_from or {}).items():
        b.instance(i).match_energy(b.instance(j).poll()["energy"])
    b.autotune(reps=3)
    t0 = time.perf_counter()
    done = 0
    probe_res = None
    hist = []
    while done < cap:
        n = min(probe if (probe and done == 0) else chunk, cap - done)
        b.run(tol=tol, consecutive=3, poll_every=poll, max_steps=n, allow_unstable=True)
        done += n
        st = b.status()
        if trace:
            hist.append((done, st["residual"].copy()))
        if probe and probe_res is None:
            probe_res = st["residual"].copy()
        log(f"  {time.perf_counter() - t0:.0f} s, {done} steps: {int((st['state'] != 0).sum())}/{len(fields)} retired")
        if (st["state"] != 0).all():
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = b.status()
    if probe_res is not None:
        st["probe_residual"] = probe_res
    if trace:
        st["trace"] = hist
    out = []
    for i in range(len(fields)):
        (rho, _, _, T), _ = b.instance(i).moments(globals_=False)
        out.append((rho.cpu().numpy(), T.cpu().numpy()))
    b.close()
    return st, out, wall


def instances(n, seed, size):
    return W.batch_instances(n, seed=seed, sizes=(size,))


def network_input(rho0, T0, t_ratio):
    return np.stack([rho0 / W.RHO_CRIT, T0 / W.T_CRIT, np.full_like(rho0, t_ratio)]).astype(np.float32)


def make_dataset(n, seed, size, tol, cap, per_batch=64):
    xs, ys, steps = [], [], []
    for first in range(0, n, per_batch):
        inst = instances(min(per_batch, n - first), seed + first, size)
        log(f"relaxing instances {first}..{first + len(inst) - 1}")
        fields = [(f.rho, f.ux, f.uy, f.T) for _, _, _, _, f in inst]
        st, relaxed, _ = run_batch(fields, tol, cap)
        for (kind, Nn, t, R, f), (rho, T), s in zip(inst, relaxed, st["steps"]):
            xs.append(network_input(f.rho, f.T, t))
            ys.append(np.stack([rho / W.RHO_CRIT, T / W.T_CRIT]).astype(np.float32))
            steps.append(int(s))
    return np.stack(xs), np.stack(ys), steps


def train(x, y, epochs, batch, lr, seed=0, net=None):
    h, w = x.shape[2], x.shape[3]
    if net is None:
        net = N.Network(h, w, batch, torch.from_numpy(W.cnn_init_params(seed)))
    dev = net.device
    X = torch.from_numpy(x).to(dev)
    Y = torch.from_numpy(y).to(dev)
    rng = np.random.default_rng(seed)
    hist = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = rng.permutation(len(x))
        losses = []
        for i in range(0, len(x) - batch + 1, batch):
            idx = torch.from_numpy(perm[i:i + batch]).to(dev)
            # cosine decay of the learning rate over the run
            frac = (ep + i / len(x)) / epochs
            L = net.train_step(X.index_select(0, idx), Y.index_select(0, idx), lr * 0.5 * (1 + np.cos(np.pi * frac)))
            losses.append(L)
        hist.append(float(torch.stack(losses).mean()))
        if ep % max(1, epochs // 10) == 0 or ep == epochs - 1:
            log(f"  epoch {ep}: loss {hist[-1]:.3e}")
    torch.cuda.synchronize()
    return net, hist, time.perf_counter() - t0


def decay_fit(steps, resid, lo, hi):
    """Exponential fit r = r0 exp(-lam s) of a residual history over the points with
    lo < r < hi (the tail before retirement): (r0, lam) or None with fewer than 3 points."""
    sel = [(s, r) for s, r in zip(steps, resid) if lo < r < hi]
    if len(sel) < 3:
        return None
    s_, r_ = np.array(sel, dtype=np.float64).T
    slope, icpt = np.polyfit(s_, np.log(r_), 1)
    return float(np.exp(icpt)), float(-slope)


def evaluate(net, n, seed, size, tol, cap, probe=1000, chunk=5000, precision=0):
    """Cold and warm runs of n held-out instances in one batch; steps to tolerance, and the
    best-of-two start decided by the residuals after `probe` steps.  Also, per instance: the
    RMS distance of each start from the relaxed cold field (normalised by rho_c) and the
    exponential decay of each run's residual (fitted between 10 tol and 1e-5)."""
    inst = instances(n, seed, size)
    cold, warm, infer = [], [], []
    for kind, Nn, t, R, f in inst:
        cold.append((f.rho, f.ux, f.uy, f.T))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rho, T = net.warm_start(torch.from_numpy(f.rho), torch.from_numpy(f.T), t * W.T_CRIT, W.RHO_CRIT, W.T_CRIT,
                                0.95 / W.EOS_B)
        torch.cuda.synchronize()
        infer.append(time.perf_counter() - t0)
        r, Tn = rho.cpu().numpy(), T.cpu().numpy()
        warm.append((r, np.zeros_like(r), np.zeros_like(r), Tn))
    # the warm starts take the total energy of their cold starts (mass is kept by the transform)
    st, relaxed, wall = run_batch(cold + warm, tol, cap, chunk=chunk, probe=probe,
                                  energy_from={n + k: k for k in range(n)}, trace=True, precision=precision)
    s = st["steps_to_tol"]
    sc, sw = s[:n], s[n:]
    ok = (sc > 0) & (sw > 0)
    # best of two: both starts run `probe` steps, the one with the smaller residual
    # continues; its cost counts the other start's probe steps as well
    rp = st["probe_residual"]
    pick_warm = rp[n:] < rp[:n]
    sch = np.where(pick_warm, sw, sc)
    sb = np.where(sch > 0, sch + probe, -1)
    # relaxed states of the two starts of each instance: how far apart they end
    diff = [float(np.abs(relaxed[i][0] - relaxed[n + i][0]).max()) for i in range(n)]
    # distance of each start from the relaxed cold field, and the residual decay of each run
    err_cold = [float(np.sqrt(np.mean((cold[i][0] - relaxed[i][0]) ** 2)) / W.RHO_CRIT) for i in range(n)]
    err_warm = [float(np.sqrt(np.mean((warm[i][0] - relaxed[i][0]) ** 2)) / W.RHO_CRIT) for i in range(n)]
    tsteps = [h[0] for h in st["trace"]]
    fits = [decay_fit(tsteps, [h[1][i] for h in st["trace"]], 10 * tol, 1e-5) for i in range(2 * n)]
    kinds = [(k, float(t), float(R)) for k, _, t, R, _ in inst]
    return {"instances": n, "tol": tol, "cap": cap, "precision": precision, "both_converged": int(ok.sum()),
            "cold_capped": int((sc < 0).sum()), "warm_capped": int((sw < 0).sum()),
            "steps_cold_median": float(np.median(np.where(sc > 0, sc, cap))),
            "steps_warm_median": float(np.median(np.where(sw > 0, sw, cap))),
            "speedup_median": float(np.median(np.where(sc > 0, sc, cap) / np.where(sw > 0, sw, cap))),
            "probe": probe, "best_capped": int((sb < 0).sum()), "best_picked_warm": int(pick_warm.sum()),
            "steps_best_median": float(np.median(np.where(sb > 0, sb, cap))),
            "speedup_best_median": float(np.median(np.where(sc > 0, sc, cap) / np.where(sb > 0, sb, cap))),
            "inference_ms_median": 1e3 * float(np.median(infer)),
            "final_rho_maxdiff_median": float(np.median(diff)),
            "steps_cold": [int(v) for v in sc], "steps_warm": [int(v) for v in sw],
            "steps_best": [int(v) for v in sb], "rms_start_error_cold": err_cold, "rms_start_error_warm": err_warm,
            "decay_cold": fits[:n], "decay_warm": fits[n:], "instances_kind_T_R": kinds,
            "trace_steps": tsteps, "trace_residual": [[float(v) for v in h[1]] for h in st["trace"]]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--train", type=int, default=128, help="training instances")
    ap.add_argument("--eval", type=int, default=64, help="held-out instances")
    ap.add_argument("--data-tol", type=float, default=1e-6)
    ap.add_argument("--data-cap", type=int, default=100000)
    ap.add_argument("--tol", type=float, default=3e-7)
    ap.add_argument("--cap", type=int, default=200000)
    ap.add_argument("--precision", type=int, default=0, help="state of the evaluation runs (1: compensated)")
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--save-params", help="write the trained parameters (float32 .npy)")
    ap.add_argument("--load-params", help="skip data and training: evaluate these parameters")
    args = ap.parse_args()
    out = {"size": args.size}
    if args.load_params:
        theta = np.load(args.load_params)
        net = N.Network(args.size, args.size, 1, torch.from_numpy(theta.astype(np.float32)))
        out["params"] = args.load_params
    else:
        t0 = time.perf_counter()
        x, y, steps = make_dataset(args.train, 10000, args.size, args.data_tol, args.data_cap)
        t_data = time.perf_counter() - t0
        log(f"dataset: {len(x)} samples in {t_data:.0f} s (median {np.median(steps):.0f} steps)")
        net, hist, t_train = train(x, y, args.epochs, args.batch, args.lr)
        log(f"trained in {t_train:.0f} s: loss {hist[0]:.3e} -> {hist[-1]:.3e}")
        if args.save_params:
            np.save(args.save_params, net.params.cpu().numpy())
        out.update({"train_instances": len(x), "data_tol": args.data_tol, "data_cap": args.data_cap,
                    "data_steps_median": float(np.median(steps)), "data_seconds": t_data, "epochs": args.epochs,
                    "batch": args.batch, "lr": args.lr, "train_seconds": t_train, "loss_first": hist[0],
                    "loss_last": hist[-1]})
    out["evaluation"] = evaluate(net, args.eval, 20000, args.size, args.tol, args.cap, precision=args.precision)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
