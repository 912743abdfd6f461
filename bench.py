#!/usr/bin/env python3
"""Throughput of the FFT-LB time step on one MI355X.

Workload: spinodal quench on a 1024 x 1024 periodic grid (rho = rho_c (1 + 0.005 xi),
T = 0.8 T_c, a = 2, b = 0.4, the paper's dx, dt, tau, K, q and the k4 window).  A step is
one full FFT-LB update of all 33 populations (convection and force derivatives by
windowed FFT, collision, force, moments).  Inputs are resident in HBM when timing starts.

Prints one JSON line.  value = site-velocity updates per second = 33 nx ny steps / s.
roofline: the dominant kernel's algorithmic bytes per launch over its mean launch time,
timed with HIP events on the stream it runs on, against 8 TB/s.
batch: the 64-instance batched workload's throughput; time_to_equilibrium: steps and wall
time of a batch of instances (compensated state) to the residual 1e-8.
cpu_baseline: the FP64 oracle timed on this host's cores (a bounded sample of the same
workload, plus the 64^2 and 256^2 configurations and a single-core figure).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "site·velocity updates/s per FFT-LB step; % HBM roofline; time-to-equilibrium"

# Algorithmic bytes per site of each kernel of the step (FP32 values; a packed half
# spectrum of a real plane is nx*ny/2 complex = one float per site):
# (the convection columns of the 24 populations with v_y != 0 are split 16 / 8 over the two
# derivative column launches; each reads its f plane and writes the real y-part v_y D_y f):
#   0 stage-1 + convection columns: read 4 moment spectra, write 6 y-derivatives,
#                         read and write 16 population planes             ->  42 floats
#   1 stage-2 rows:       read 4 + 6 spectra + 4 fields, write 5 spectra + C -> 20
#   2 stage-2 + convection columns: read 5 spectra, write 3,
#                         read and write 8 population planes              ->  24
#   3 collide rows:       read f (33) + 24 y-parts + 3 + C + 4 fields,
#                         write f (33) + 4 moment spectra + 4 fields       -> 106
#                         (the x-parts v_x D_x f are formed from f^n in the kernel: no
#                         population spectra are stored or read)
STAGES = ("stage1_conv_columns", "stage2_rows", "stage2_conv_columns", "collide_rows")
STAGE_KERNELS = ("k_col_conv_multi", "k_rows_stage2", "k_col_conv_multi", "k_rows_collide")
STAGE_FLOATS_PER_SITE = (42, 20, 24, 106)
DOMINANT = 3

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_collide_spinodal1024.json")
CSRC = os.path.join(ROOT, "paper_1011_3582_amd", "csrc")


def _code_only(text: bytes) -> bytes:
    """Source text without its comments and with whitespace collapsed."""
    text = re.sub(rb"/\*.*?\*/", b" ", text, flags=re.S)
    text = re.sub(rb"//[^\n]*", b" ", text)
    return b" ".join(text.split())


def kernel_source_hash() -> str:
    """Hash of the code of every source the solver's kernels are built from: the device
    headers and the translation units that instantiate the kernels (the host API, fftlb.hip,
    and the warm-start network's files excluded).  Comments and layout do not count."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if (name.endswith(".hpp") or name.startswith(("rows_", "cols_"))) and not name.startswith("cnn."):
            with open(os.path.join(CSRC, name), "rb") as fh:
                h.update(name.encode() + _code_only(fh.read()))
    return h.hexdigest()[:16]


def measured_traffic(nx, ny):
    """HBM bytes per launch of the dominant kernel from committed rocprofv3 counter runs,
    scaled by the copy-kernel calibration; None if absent or taken on other kernel code."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash() or rec.get("nx") != nx or rec.get("ny") != ny:
        return None
    return rec.get("bytes_per_launch")


def write_traffic(fetch_csv, write_csv, calib_mib, nx, ny):
    """Turn two rocprofv3 --pmc counter files (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) of
    a run with --calib-copy-mib into the dominant kernel's HBM bytes per launch.  Each
    counter is scaled by what it reads for the largest plain device copy of the same run
    (calib_mib MiB read and written)."""
    import csv
    import statistics

    def per_kernel(path, counter):
        vals = {}
        for row in csv.DictReader(open(path)):
            if row["Counter_Name"] == counter:
                vals.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
        return vals

    # the step's collide: MODE_STEP, FP32 state, population spectra of the windowed path
    want = f"{STAGE_KERNELS[DOMINANT]}<{nx}, 0, false, false>"
    rec = {"source_hash": kernel_source_hash(), "nx": nx, "ny": ny, "kernel": want,
           "calib_copy_kib": calib_mib * 1024}
    total = 0.0
    for key, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        vals = per_kernel(path, key)
        copy = max(v for k, vs in vals.items() if "copyBuffer" in k for v in vs)
        scale = calib_mib * 1024 / copy
        mine = [v for k, vs in vals.items() if want in k for v in vs]
        if not mine:
            raise SystemExit(f"no dispatch of {want} in {path}")
        kib = statistics.mean(mine)
        rec[key] = {"kib_per_dispatch": kib, "dispatches": len(mine), "copy_kib": copy, "scale": scale}
        total += kib * scale * 1024
    rec["bytes_per_launch"] = total
    rec["algorithmic_bytes_per_launch"] = STAGE_FLOATS_PER_SITE[DOMINANT] * 4 * nx * ny
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def batch_leg(args, F, W, dev):
    """64 independent instances of uneven grid sizes (128..512 squared; droplets and slabs at
    0.80..0.98 T_c) advanced together: aggregate site-velocity updates per second over
    `--batch-steps` steps (residual tolerance 0, nothing retires)."""
    import torch
    inst = W.batch_instances(64, seed=3)
    fields = [tuple(torch.from_numpy(a) for a in (f.rho, f.ux, f.uy, f.T)) for _, _, _, _, f in inst]
    sites = sum(N * N for _, N, _, _, _ in inst)
    print(f"[bench] batch: {len(inst)} instances, {sites} sites", file=sys.stderr, flush=True)
    b = F.Batch(fields, device=dev)
    if not args.no_autotune:
        b.autotune(reps=5)
    b.run(tol=0.0, poll_every=100, max_steps=100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(tol=0.0, poll_every=100, max_steps=args.batch_steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    steps = int(b.status()["steps"][0]) - 100
    plans = {}
    for i, (_, N, _, _, _) in enumerate(inst):
        plans.setdefault(str(N), list(b.instance(i).plan))
    b.close()
    return {"workload": "64 instances, N x N with N uniform over {128, 192, 256, 384, 512}, T/Tc uniform over "
                        "0.80..0.98, droplet (R 10..60) or slab, tanh width 4 (seed 3)",
            "instances": len(inst), "sites": sites, "steps": steps, "ms_per_step": wall / steps * 1e3,
            "value": 33.0 * sites * steps / wall, "unit": "site·velocity updates/s", "plans": plans}


def equilibrium_leg(F, W, dev, n, sizes, tol, cap, seed=3):
    """Time to equilibrium: n instances of the batched workload (grid sizes `sizes`) with the
    compensated state (precision 1: increments below half an FP32 ulp accumulate, so the
    residual can fall below the FP32 state's floor of about 4e-8..1e-7), run until each one's
    residual dt max|D.(rho u)| (= max |rho^{n+1} - rho^n|) stays below tol at 3 polls 100
    steps apart, or `cap` steps."""
    import numpy as np
    import torch
    inst = W.batch_instances(n, seed=seed, sizes=sizes)
    fields = [tuple(torch.from_numpy(a) for a in (f.rho, f.ux, f.uy, f.T)) for _, _, _, _, f in inst]
    sites = sum(N * N for _, N, _, _, _ in inst)
    print(f"[bench] time to residual {tol:g}: {n} instances ({sites} sites), cap {cap} steps",
          file=sys.stderr, flush=True)
    b = F.Batch(fields, F.Params(precision=1), device=dev)
    b.autotune(reps=3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < cap:
        chunk = min(20000, cap - done)
        b.run(tol=tol, consecutive=3, poll_every=100, max_steps=chunk, allow_unstable=True)
        done += chunk
        st = b.status()
        print(f"[bench]   {time.perf_counter() - t0:.0f} s, {done} steps: {int((st['state'] != 0).sum())}/{n} "
              f"retired, median residual {np.median(st['residual']):.2e}", file=sys.stderr, flush=True)
        if (st["state"] != 0).all():
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = b.status()
    b.close()
    conv = st["steps_to_tol"][st["state"] == 1]
    per = [{"kind": k, "N": N, "T/Tc": t, "R": R, "steps_to_tol": int(s)}
           for (k, N, t, R, _), s in zip(inst, st["steps_to_tol"])]
    return {"workload": f"{n} instances of the batched workload with N in {list(sizes)} (seed {seed}), "
                        "compensated FP32 state", "tol": tol, "cap": cap, "sites": sites, "wall_s": wall,
            "converged": int(len(conv)), "unstable": int((st["state"] == 2).sum()),
            "capped": int((st["state"] == 0).sum()),
            "steps_to_tol": {"min": int(conv.min()) if len(conv) else None,
                             "median": float(np.median(conv)) if len(conv) else None,
                             "max": int(conv.max()) if len(conv) else None},
            "instances": per}


def cpu_baseline(params, cores=None):
    """The FP64 oracle, as it stands, timed on this host: the 1024 x 1024 quench (one warm-up
    step, then 2 steps on all the host cores given to this process (at most 16, the CPU share
    of one GPU) and 1 step on one core), and, on all cores, the 64 x 64 slab (30 steps after
    one) and the 256 x 256 droplet (4 steps after one).  About 15 s of CPU work."""
    import numpy as np
    import scipy
    from oracle import fftlb_oracle as O
    from paper_1011_3582_amd import workloads as W
    avail = len(os.sched_getaffinity(0))
    cores = cores or min(16, avail)
    op = O.Params(dx=params.dx, dy=params.dy, dt=params.dt, tau=params.tau, K=params.K, H=params.H,
                  zeta=params.zeta, q=params.q, a=params.a, b=params.b, m=params.m)

    def rate(fields, steps, workers, warmup):
        f = O.feq(*fields.as_f64())
        for _ in range(warmup):
            f = O.step(f, op, workers=workers)
        t0 = time.perf_counter()
        for _ in range(steps):
            f = O.step(f, op, workers=workers)
        dt = (time.perf_counter() - t0) / steps
        return 33.0 * f.shape[1] * f.shape[2] / dt, dt

    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    spin = W.spinodal_1024()
    v_all, t_all = rate(spin, 2, cores, 1)
    v_one, t_one = rate(spin, 1, 1, 0)
    v64, t64 = rate(W.slab_64(), 30, cores, 1)
    v256, t256 = rate(W.droplet_256(), 4, cores, 1)
    return {"value": v_all, "unit": "site·velocity updates/s", "cores": cores, "kind": "oracle",
            "sample": f"2 steps of the 1024x1024 quench after 1 warm-up step, FP64 NumPy/SciPy (pocketfft, "
                      f"{cores} workers): {t_all:.2f} s per step",
            "single_core": {"value": v_one, "s_per_step": t_one},
            "host": {"cpu": model, "cpus_available": avail, "numpy": np.__version__, "scipy": scipy.__version__},
            "configs": {"slab 64x64 (30 steps)": {"value": v64, "s_per_step": t64},
                        "droplet 256x256 (4 steps)": {"value": v256, "s_per_step": t256}}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=32)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default column plan")
    ap.add_argument("--batch-steps", type=int, default=200,
                    help="timed steps of the 64-instance batch (0: skip the batch leg)")
    ap.add_argument("--equilibrium-tol", type=float, default=1e-8, metavar="TOL",
                    help="residual tolerance of the time-to-equilibrium leg (the batched workload's 1e-8)")
    ap.add_argument("--equilibrium-instances", type=int, default=16,
                    help="instances of the time-to-equilibrium leg (0: skip it)")
    ap.add_argument("--equilibrium-sizes", default="128,192",
                    help="grid sizes of the time-to-equilibrium leg (comma separated)")
    ap.add_argument("--equilibrium-cap", type=int, default=400_000)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this size (traffic calibration under rocprofv3)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic record from two rocprofv3 counter files and exit")
    args = ap.parse_args()
    if args.traffic_from:
        write_traffic(*args.traffic_from, args.calib_copy_mib or 1024, 1024, 1024)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1011_3582_amd import fftlb as F
    from paper_1011_3582_amd import workloads as W

    nx = ny = 1024
    fields = W.spinodal_1024()
    params = F.Params()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    s = F.Solver(*(torch.from_numpy(a) for a in (fields.rho, fields.ux, fields.uy, fields.T)), params, device=dev)
    plan = s.plan
    if not args.no_autotune:
        print("[bench] autotune column plans", file=sys.stderr, flush=True)
        plan = s.autotune(reps=10)
    print(f"[bench] warmup {args.warmup} steps", file=sys.stderr, flush=True)
    s.step(args.warmup)
    torch.cuda.synchronize()

    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    s.step(args.steps)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_s = ev0.elapsed_time(ev1) / 1e3
    _, glob = s.moments()
    assert glob["nonfinite"] == 0.0, "state became non-finite"

    # per-kernel mean launch time, HIP events on the stream the kernels run on
    state = s.get_state()
    kern_ms = []
    for k in range(len(STAGES)):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.run_stage(k, 2)
        a.record()
        s.run_stage(k, args.kernel_reps)
        b.record()
        torch.cuda.synchronize()
        kern_ms.append(a.elapsed_time(b) / args.kernel_reps)
        s.set_state(state)
    s.close()

    batch = batch_leg(args, F, W, dev) if args.batch_steps > 0 else None
    equil = None
    if args.equilibrium_instances > 0:
        sizes = tuple(int(v) for v in args.equilibrium_sizes.split(","))
        equil = equilibrium_leg(F, W, dev, args.equilibrium_instances, sizes, args.equilibrium_tol,
                                args.equilibrium_cap)

    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()

    # context for the roofline fraction: what a plain device copy (torch) reaches on this GPU
    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(10):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 2.0 * (1 << 30) * 10 / (c0.elapsed_time(c1) / 1e3) / 1e9
    del src, dst

    sites = nx * ny
    step_s = wall / args.steps
    value = 33.0 * sites * args.steps / wall
    t_dom = kern_ms[DOMINANT] / 1e3
    bytes_dom = STAGE_FLOATS_PER_SITE[DOMINANT] * 4 * sites
    achieved = bytes_dom / t_dom / 1e9
    traffic = measured_traffic(nx, ny)
    step_bytes = sum(STAGE_FLOATS_PER_SITE) * 4 * sites
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "site·velocity updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "spinodal quench 1024x1024 (rho_c(1+0.005 xi), T=0.8 Tc, a=2, b=0.4, "
                               "dx=1/256, dt=1e-5, tau=1e-2, K=1e-5, q=-0.004, k4 window)",
                   "nx": nx, "ny": ny, "precision": "FP32 step, FP64 global reductions"},
        "roofline": {"bound": "hbm", "kernel": STAGE_KERNELS[DOMINANT], "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "bytes_per_launch": bytes_dom, "launch_ms": kern_ms[DOMINANT]},
        "step_roofline": {"bytes_per_step": step_bytes, "achieved_GBs": step_bytes / step_s / 1e9,
                          "frac": step_bytes / step_s / 1e9 / HBM_PEAK_GBS,
                          "kernel_ms": dict(zip(STAGES, kern_ms)),
                          "event_ms_per_step": ev_s / args.steps * 1e3},
        "device_copy": {"GBs": copy_gbs, "bytes": 2 * (1 << 30),
                        "note": "torch device-to-device copy of 1 GiB (read + write), for context"},
        "globals": {k: glob[k] for k in ("mass", "energy", "residual", "umax")},
        "plan": {"conv_cols": plan[0], "multi_cols": plan[1], "conv_radix": plan[2], "multi_radix": plan[3]},
    }
    if batch is not None:
        out["batch"] = batch
    if equil is not None:
        out["time_to_equilibrium"] = equil
    if not args.no_cpu_baseline:
        print("[bench] oracle CPU baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(params)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
