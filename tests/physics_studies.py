"""Physics studies of the FFT-LB step at the paper's equation-of-state constants (a = 9/8,
b = 1/3, T_c = rho_c = 1): runs on the GPU through the library (paper_1011_3582_amd.validation),
references from the van der Waals free energy (oracle/thermo.py).  Test infrastructure: the
GPU tests in test_gpu_physics.py call shorter versions; the full studies write the summaries
under profiles/.

  laplace(): droplets of several radii at T = 0.95 for K = 1e-5, 7.5e-6, 5e-6 relax in one
      batch; the pressure jump dP = P_in - P_out (P_in the mean bulk pressure over the sites
      within R/2 of the centre, P_out over those beyond 3R/2, Sec. 4.2) against 1/R gives the
      surface tension as the slope (Laplace law, Eq. (55)), compared with
      sigma = K int (d rho/dz)^2 dz of the planar equilibrium interface (Eq. (56));
  profile(): a relaxed planar slab against the equilibrium profile of the square-gradient
      model (the interface integral of Eqs. (51)-(53));
  coexistence(): slabs started with the densities of a temperature 0.02 T_c higher than
      their own relax to the coexistence curve of the Maxwell construction (Sec. 4.1, the
      temperature steps of the coexistence-curve study);
  energy(): Delta e_T of the phase separation for k1..k4 and exact k (or any window orders and
      finite-difference schemes), also measured with one common (exact-gradient) energy
      definition;
  spurious(): the spurious velocities of planar interfaces (Sec. 4.1, the paper's Figs. 10, 12
      and 14) for the k4 window and the finite-difference schemes (NPS, MLW2, LW, CD), with the
      bulk densities against the Maxwell construction;
  droplet_currents(): the spurious currents of a circular droplet started at equilibrium
      (Sec. 4.2, Fig. 19) for k1..k4, NPS and CD;
  slab_floor(): the spurious velocity of an equilibrium slab at K = 1e-5 with f in FP32, with the
      compensated state and (optionally) in the FP64 oracle;
  cooling(): the paper's coexistence protocol, a slab cooled from 0.97 T_c in steps of 0.02, per
      discretisation.

Usage (one MI355X):
  python tests/physics_studies.py laplace|profile|coexistence|energy|spurious [--cap N] [--orders ...]
"""
import argparse
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import thermo  # noqa: E402
from paper_1011_3582_amd import fftlb as F  # noqa: E402
from paper_1011_3582_amd import validation as V  # noqa: E402

A, B = 9.0 / 8.0, 1.0 / 3.0
log = V.log


def laplace(n=192, radii=(24, 28, 32, 36, 40), Ks=(1e-5, 7.5e-6, 5e-6), t_ratio=0.95, tol=1e-9, cap=1_000_000):
    T = t_ratio * 8 * A / (27 * B)
    fields, params, keys = [], [], []
    for K in Ks:
        p = F.Params(a=A, b=B, K=K, precision=1)
        for R in radii:
            fields.append(V.droplet_from_profile(n, R, lambda s, K=K: thermo.planar_profile(s, T, A, B, K), T, p.dx))
            params.append(p)
            keys.append((K, R))
    dx = F.Params().dx
    history = []

    def fits(relaxed):
        out = {}
        for K in Ks:
            sel = [i for i, (k, _) in enumerate(keys) if k == K]
            inv_r = [1.0 / (V.equimolar_radius(relaxed[i][0]) * dx) for i in sel]
            dps = [V.pressure_jump(relaxed[i][0], relaxed[i][1], V.equimolar_radius(relaxed[i][0])) for i in sel]
            out[K] = np.polyfit(inv_r, dps, 1)
        return out

    def monitor(steps, relaxed):
        f = fits(relaxed)
        history.append({"steps": steps, "sigma_fit": {f"{K:g}": float(f[K][0]) for K in Ks}})
        log("  sigma fits " + ", ".join(f"{K:g}: {f[K][0]:.4e}" for K in Ks))

    st, relaxed = V.relax(fields, params, tol, cap, label="laplace", monitor=monitor)
    res = {"n": n, "T/Tc": t_ratio, "tol": tol, "cap": cap, "history": history, "K": {}}
    for K in Ks:
        inv_r, dps, rows = [], [], []
        for (k, R0), (rho, Tf), steps, state, resid in zip(keys, relaxed, st["steps"], st["state"], st["residual"]):
            if k != K:
                continue
            Req = V.equimolar_radius(rho)
            dp = V.pressure_jump(rho, Tf, Req)
            inv_r.append(1.0 / (Req * dx))
            dps.append(dp)
            rows.append({"R0": R0, "R_equimolar": Req, "dP": dp, "T_mean": float(Tf.mean()), "steps": int(steps),
                         "state": int(state), "residual": float(resid)})
        slope, intercept = np.polyfit(inv_r, dps, 1)
        t_end = float(np.mean([r["T_mean"] for r in rows]))
        sigma = thermo.surface_tension(t_end, A, B, K)
        res["K"][f"{K:g}"] = {"sigma_fit": float(slope), "intercept": float(intercept), "sigma_theory": sigma,
                              "rel_err": abs(slope - sigma) / sigma, "T_end": t_end, "droplets": rows}
        log(f"K {K:g}: sigma fit {slope:.4e}, theory {sigma:.4e} (T {t_end:.5f}), intercept {intercept:.2e}")
    return res


def coexistence(temps=(0.80, 0.82, 0.84, 0.86, 0.88, 0.90, 0.92, 0.94, 0.96, 0.98), step=0.02, nx=256, ny=4,
                tol=1e-10, cap=1_000_000):
    """Slabs (liquid in nx/4 < x <= 3nx/4) at T, started from the coexistence densities of T + step
    (tanh interfaces of the equilibrium width at T + step): the bulk densities must move to
    the coexistence curve at the relaxed temperature."""
    t_c = 8 * A / (27 * B)
    fields, params = [], []
    x = np.arange(nx, dtype=np.float64)
    for tr in temps:
        p = F.Params(a=A, b=B, precision=1)
        hot = min(tr + step, 0.995) * t_c
        dist = np.minimum(x - nx / 4.0, 3.0 * nx / 4.0 - x) * p.dx
        fields.append(V.slab_start(nx, ny, thermo.planar_profile(dist, hot, A, B, p.K), tr * t_c))
        params.append(p)
    history = []

    def monitor(steps, relaxed):
        row = {"steps": steps, "gap_error": []}
        for (rho, T) in relaxed:
            rv, rl = V.bulk_densities(rho)
            mv, ml = thermo.maxwell(float(T.mean()), A, B)
            row["gap_error"].append(max(abs(rv - mv), abs(rl - ml)) / (ml - mv))
        history.append(row)
        log("  worst distance to the curve (of the gap): " + f"{max(row['gap_error']):.2e}")

    st, relaxed = V.relax(fields, params, tol, cap, label="coexistence", monitor=monitor)
    rows = []
    for tr, (rho, T), steps, state in zip(temps, relaxed, st["steps"], st["state"]):
        rv, rl = V.bulk_densities(rho)
        t_end = float(T.mean())
        mv, ml = thermo.maxwell(t_end, A, B)
        sv, sl = thermo.maxwell(min(tr + step, 0.995) * t_c, A, B)
        rows.append({"T/Tc": tr, "T_end": t_end, "rho_v": rv, "rho_l": rl, "maxwell_v": mv, "maxwell_l": ml,
                     "start_v": sv, "start_l": sl, "gap_error": max(abs(rv - mv), abs(rl - ml)) / (ml - mv),
                     "start_gap_error": max(abs(sv - mv), abs(sl - ml)) / (ml - mv), "steps": int(steps),
                     "state": int(state)})
    return {"nx": nx, "ny": ny, "step": step, "tol": tol, "cap": cap, "slabs": rows, "history": history}


def profile(t_ratio=0.95, K=1e-5, nx=256, ny=4, start_width=2.0, tol=1e-10, cap=400_000):
    """A slab started from the equilibrium profile stretched by start_width (a non-equilibrium
    interface) relaxes; the relaxed profile is compared with the equilibrium profile of the
    square-gradient model at the relaxed temperature, centred at the relaxed interface."""
    t_c = 8 * A / (27 * B)
    T = t_ratio * t_c
    p = F.Params(a=A, b=B, K=K, precision=1)
    x = np.arange(nx, dtype=np.float64)
    dist = np.minimum(x - nx / 4.0, 3.0 * nx / 4.0 - x) * p.dx
    start = thermo.planar_profile(dist / start_width, T, A, B, K)
    st, relaxed = V.relax([V.slab_start(nx, ny, start, T)], [p], tol, cap, label="profile")
    rho, Tf = relaxed[0]
    prof = rho.mean(axis=0)
    t_end = float(Tf.mean())
    mv, ml = thermo.maxwell(t_end, A, B)
    # interface positions: where the profile crosses the mid density (linear interpolation)
    mid = 0.5 * (prof[:nx // 2].min() + prof[nx // 4: 3 * nx // 4].max())
    i = int(np.argmax(prof[: nx // 2] > mid))
    x0 = i - 1 + (mid - prof[i - 1]) / (prof[i] - prof[i - 1])
    theory = thermo.planar_profile((x - x0) * p.dx, t_end, A, B, K)
    win = slice(int(x0) - 24, int(x0) + 25)
    err = np.abs(prof[win] - theory[win]).max() / (ml - mv)
    start_err = np.abs(start[win] - thermo.planar_profile((x[win] - nx / 4) * p.dx, T, A, B, K)).max()
    return {"T/Tc": t_ratio, "K": K, "nx": nx, "start_width_factor": start_width, "T_end": t_end,
            "interface_x": x0, "max_err_of_gap": float(err), "start_max_err_of_gap": float(start_err / (ml - mv)),
            "steps": int(st["steps"][0]), "state": int(st["state"][0]), "residual": float(st["residual"][0]),
            "profile": [float(v) for v in prof[win]], "theory": [float(v) for v in theory[win]]}


def energy(cap=500_000, orders=(1, 2, 3, 4, 0)):
    """Delta e_T of the 128 x 128 phase separation (paper_1011_3582_amd.validation.energy) for each
    window, as each run measures it (its own windowed gradient in K |grad rho|^2 / 2) and with one
    common definition: the energy of Eq. (17) of the initial and final macroscopic fields with the
    exact spectral gradient (oracle.fftlb_oracle.fields_energy, m = 0), so that the windows are
    compared on the same quantity."""
    from oracle import fftlb_oracle as O
    res = V.energy(cap=cap, orders=orders, keep_fields=True)
    kept = res.pop("fields")
    n = res["n"]
    p = F.Params(a=A, b=B)
    area = n * n * p.dx * p.dy

    def e_exact(fields):
        op = O.Params(dx=p.dx, dy=p.dy, dt=p.dt, tau=p.tau, K=p.K, H=p.H, zeta=p.zeta, q=p.q, a=A, b=B, m=0)
        return O.fields_energy(*fields, op) / area

    e0 = e_exact(kept["initial"])
    res["de_T_exact_gradient"] = {k: e_exact(v) - e0 for k, v in kept.items() if k != "initial"}
    res["gradient_energy_final"] = {}
    for k, (rho, ux, uy, T) in kept.items():
        if k == "initial":
            continue
        op = O.Params(dx=p.dx, dy=p.dy, dt=p.dt, tau=p.tau, K=p.K, H=p.H, zeta=p.zeta, q=p.q, a=A, b=B, m=0)
        D = O.Deriv(n, n, op)
        res["gradient_energy_final"][k] = float((0.5 * p.K * (D.x(rho) ** 2 + D.y(rho) ** 2)).mean())
    log("Delta e_T (own window): " + ", ".join(f"{k}: {v:.4e}" for k, v in res["final_de_T"].items()))
    log("Delta e_T (exact gradient): " + ", ".join(f"{k}: {v:.4e}" for k, v in res["de_T_exact_gradient"].items()))
    return res


def spurious(cases=((0.93, 0.0), (0.93, 5e-6), (0.85, 5e-6)), orders=(4, "NPS+NPS", "MLW2+CD", "LW+CD", "CD+CD"),
             nx=512, ny=4, cap=1_000_000, every=50_000):
    """Planar interfaces (Sec. 4.1): slabs with liquid in nx/4 < x <= 3nx/4 at each (T/T_c, K) of
    `cases`, started at the Maxwell coexistence densities of T with the equilibrium profile
    (K > 0) or a tanh of width 1.5 grid units (K = 0, where the equilibrium interface is sharp),
    u = 0; every case with every discretisation in one batch for cap steps.  u^s = max |u|
    against time, the final u_x(x) (mean over y) and the bulk densities against Maxwell's."""
    t_c = 8 * A / (27 * B)
    x = np.arange(nx, dtype=np.float64)
    dist = np.minimum(x - nx / 4.0, 3.0 * nx / 4.0 - x)   # grid units, > 0 in the liquid
    fields, params, keys = [], [], []
    for tr, K in cases:
        T = tr * t_c
        mv, ml = thermo.maxwell(T, A, B)
        dx = F.Params().dx
        prof = (thermo.planar_profile(dist * dx, T, A, B, K) if K > 0
                else 0.5 * (ml + mv) + 0.5 * (ml - mv) * np.tanh(dist / 1.5))
        for spec in orders:
            m, conv = V.scheme(spec)
            fields.append(V.slab_start(nx, ny, prof, T))
            params.append(F.Params(a=A, b=B, K=K, m=m, convection=conv, precision=1))
            keys.append((tr, K, V.scheme_name(spec)))
    b = F.Batch([tuple(torch_from(a) for a in f) for f in fields], params)
    series = [[] for _ in keys]

    def record(steps):
        for i in range(len(keys)):
            try:
                series[i].append((steps * params[i].dt, b.instance(i).poll()["umax"]))
            except F.FFTLBError:
                series[i].append((steps * params[i].dt, None))
        if steps % (4 * every) == 0:
            log(f"spurious {steps} steps: " + ", ".join(f"{k[2]}@{k[0]},{k[1]:g}: {s[-1][1]}" for k, s in
                                                        zip(keys, series)))

    V._chunked(b, len(keys), cap, every, record)
    rows = []
    for i, (tr, K, name) in enumerate(keys):
        row = {"T/Tc": tr, "K": K, "scheme": name, "umax": series[i][-1][1],
               "umax_series": series[i]}
        if row["umax"] is not None:
            (rho, ux, _, T), _ = b.instance(i).moments(globals_=False)
            rho = rho.cpu().numpy().astype(np.float64)
            ux = ux.cpu().numpy().astype(np.float64).mean(axis=0)
            t_end = float(T.cpu().numpy().astype(np.float64).mean())
            rv, rl = V.bulk_densities(rho)
            mv, ml = thermo.maxwell(t_end, A, B)
            row.update({"T_end": t_end, "rho_v": rv, "rho_l": rl, "maxwell_v": mv, "maxwell_l": ml,
                        "ux_profile": ux.tolist(), "ux_argmax": int(np.argmax(np.abs(ux)))})
        rows.append(row)
    b.close()
    return {"nx": nx, "ny": ny, "steps": cap, "cases": rows}


def droplet_currents(n=128, R=24.0, t_ratio=0.95, K=1e-5, orders=(1, 2, 3, 4, "NPS+NPS", "CD+CD"),
                     cap=3_000_000, every=100_000):
    """The spurious currents of a circular interface (Sec. 4.2, Figs. 18-19) without the relaxation
    flow of a deformed start: a droplet of radius R (grid units) started from the planar
    equilibrium profile at T (rho = 1.46 / 0.58 is the paper's triangle at T = 0.95), u = 0, run
    for cap steps with each discretisation; u^s_max against time."""
    T = t_ratio * 8 * A / (27 * B)
    dx = F.Params().dx
    prof = lambda s_, K=K: thermo.planar_profile(s_, T, A, B, K)
    fields, params = [], []
    for spec in orders:
        m, conv = V.scheme(spec)
        fields.append(V.droplet_from_profile(n, R, prof, T, dx))
        params.append(F.Params(a=A, b=B, K=K, m=m, convection=conv, precision=1))
    b = F.Batch([tuple(torch_from(a) for a in f) for f in fields], params)
    series = [[] for _ in orders]

    def record(steps):
        for i in range(len(orders)):
            try:
                series[i].append((steps * params[i].dt, b.instance(i).poll()["umax"]))
            except F.FFTLBError:
                series[i].append((steps * params[i].dt, None))
        if steps % (5 * every) == 0:
            log(f"droplet {steps} steps: " + ", ".join(f"{V.scheme_name(o)}: {s_[-1][1]}" for o, s_ in
                                                       zip(orders, series)))

    V._chunked(b, len(orders), cap, every, record)
    b.close()
    return {"n": n, "R": R, "T/Tc": t_ratio, "K": K, "steps": cap,
            "umax": {V.scheme_name(o): s_ for o, s_ in zip(orders, series)}}


def cooling(temps=(0.97, 0.95, 0.93, 0.91, 0.89, 0.87, 0.85), K=0.0, orders=(4, "NPS+NPS", "MLW2+CD", "FL+CD"),
            nx=512, ny=4, stage_steps=500_000, every=100_000):
    """The coexistence protocol of Sec. 4.1: one slab per discretisation (liquid in
    nx/4 < x <= 3nx/4), started at T = temps[0] T_c with the densities 0.80 / 1.20 the paper takes
    from T = 0.99 and a tanh of width 1.5 grid units, run stage_steps; then cooled by the next
    step of `temps` at a time (a uniform shift of T, which changes the total energy of Eq. (17) by
    the shift times the mass: fftlb_match_energy) and run again.  After each stage: bulk
    densities, mean T and u^s against the Maxwell densities at the mean T; an instance that goes
    non-finite is reported unstable from then on."""
    t_c = 8 * A / (27 * B)
    x = np.arange(nx, dtype=np.float64)
    dist = np.minimum(x - nx / 4.0, 3.0 * nx / 4.0 - x)
    prof = 1.0 + 0.2 * np.tanh(dist / 1.5)
    fields, params = [], []
    for spec in orders:
        m, conv = V.scheme(spec)
        fields.append(V.slab_start(nx, ny, prof, temps[0] * t_c))
        params.append(F.Params(a=A, b=B, K=K, m=m, convection=conv, precision=1))
    b = F.Batch([tuple(torch_from(a) for a in f) for f in fields], params)
    stages = []
    alive = [True] * len(orders)
    for k, tr in enumerate(temps):
        if k > 0:
            shift = (temps[k] - temps[k - 1]) * t_c
            for i in range(len(orders)):
                if alive[i]:
                    g = b.instance(i).poll()
                    b.instance(i).match_energy(g["energy"] + shift * g["mass"])
        V._chunked(b, len(orders), stage_steps, every, lambda n: None)
        row = {"T/Tc": tr, "schemes": {}}
        for i, spec in enumerate(orders):
            name = V.scheme_name(spec)
            try:
                g = b.instance(i).poll()
            except F.FFTLBError:
                alive[i] = False
            if not alive[i]:
                row["schemes"][name] = None
                continue
            (rho, _, _, T), _ = b.instance(i).moments(globals_=False)
            rho = rho.cpu().numpy().astype(np.float64)
            t_end = float(T.cpu().numpy().astype(np.float64).mean())
            rv, rl = V.bulk_densities(rho)
            mv, ml = thermo.maxwell(t_end, A, B)
            row["schemes"][name] = {"T_end": t_end, "rho_v": rv, "rho_l": rl, "maxwell_v": mv, "maxwell_l": ml,
                                    "umax": g["umax"]}
        log(f"cooling T/Tc {tr}: " + ", ".join(
            f"{n}: " + ("unstable" if v is None else f"{v['rho_v']:.4f}/{v['rho_l']:.4f} u {v['umax']:.1e}")
            for n, v in row["schemes"].items()))
        stages.append(row)
    b.close()
    return {"nx": nx, "ny": ny, "K": K, "stage_steps": stage_steps, "stages": stages}


def slab_floor(nx=256, ny=4, t_ratio=0.93, K=1e-5, steps=150_000, every=2500, gpu=True, oracle=False):
    """The spurious velocity of a planar interface started from the equilibrium profile (K = 1e-5:
    the paper prints 1e-12 for it, Sec. 4.1) with the k4 window: with gpu=True the GPU with f in
    FP32 and with the compensated state, with oracle=True the FP64 oracle on the CPU from the same
    (FP32-rounded) start (slow: tens of milliseconds per step).  max |u| every `every` steps."""
    from oracle import fftlb_oracle as O
    t_c = 8 * A / (27 * B)
    T = t_ratio * t_c
    dx = F.Params().dx
    x = np.arange(nx, dtype=np.float64)
    dist = np.minimum(x - nx / 4.0, 3.0 * nx / 4.0 - x) * dx
    fields = V.slab_start(nx, ny, thermo.planar_profile(dist, T, A, B, K), T)
    fields = tuple(np.asarray(a, dtype=np.float32) for a in fields)
    out = {"nx": nx, "T/Tc": t_ratio, "K": K, "steps": steps}
    if gpu:
        params = [F.Params(a=A, b=B, K=K, precision=pr) for pr in (0, 1)]
        b = F.Batch([tuple(torch_from(a) for a in fields) for _ in params], params)
        series = {"fp32": [], "compensated": []}

        def record(n):
            for i, k in enumerate(series):
                series[k].append((n, b.instance(i).poll()["umax"]))

        V._chunked(b, 2, steps, every, record)
        b.close()
        out["gpu"] = series
    if oracle:
        op = O.Params(a=A, b=B, K=K, m=4)
        f = O.init_distribution(*(a.astype(np.float64) for a in fields))
        ser = []
        for n in range(steps + 1):
            if n % every == 0:
                _, ux, uy, _ = O.moments(f)
                ser.append((n, float(np.sqrt(ux * ux + uy * uy).max())))
                log(f"oracle {n} steps: {ser[-1][1]:.3e}")
            if n < steps:
                f = O.step(f, op, workers=os.cpu_count())
        out["oracle"] = ser
    return out


def torch_from(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32))


def sod():
    """The modified Sod tube (paper_1011_3582_amd.validation.sod) against the exact Riemann
    solution of the gamma = 2 ideal gas at t = 0.2: for each window, the L1 errors of rho, u,
    p = rho T and T over |x| < 0.6, and the total variation of rho, u and T in excess of the
    exact solution's (the grid-scale Gibbs oscillations of Fig. 7 add to it; smearing does not)."""
    from oracle import riemann
    res = V.sod()
    x = np.array(res["x"])
    win = np.abs(x) < 0.6
    ex_rho, ex_u, ex_p = riemann.sample(x[win] / res["t"], 1.0, 0.0, 1.0, 0.125, 0.0, 0.0625, 2.0)
    ex_T = ex_p / ex_rho
    p_s, u_s = riemann.star_state(1.0, 0.0, 1.0, 0.125, 0.0, 0.0625, 2.0)
    out = {"t": res["t"], "star": {"p": p_s, "u": u_s}, "windows": {}}
    # exact total variations, for reference
    out["exact_TV"] = {"rho": float(np.abs(np.diff(ex_rho)).sum()), "u": float(np.abs(np.diff(ex_u)).sum()),
                       "T": float(np.abs(np.diff(ex_T)).sum())}
    dxw = res["dx"]
    for name, prof in res["profiles"].items():
        if prof is None:
            out["windows"][name] = {"unstable": True}
            continue
        r, u, T = (np.array(prof[k])[win] for k in ("rho", "u", "T"))
        p = r * T
        l1 = lambda a, b: float(np.sum(np.abs(a - b)) * dxw)
        tv = lambda a: float(np.abs(np.diff(a)).sum())
        out["windows"][name] = {"L1_rho": l1(r, ex_rho), "L1_u": l1(u, ex_u), "L1_p": l1(p, ex_p),
                                "L1_T": l1(T, ex_T), "TV_excess_rho": tv(r) - tv(ex_rho),
                                "TV_excess_u": tv(u) - tv(ex_u), "TV_excess_T": tv(T) - tv(ex_T),
                                "umax_final": res["umax"][name][-1][1]}
        log(f"sod {name}: L1 rho {out['windows'][name]['L1_rho']:.3e}, u {out['windows'][name]['L1_u']:.3e}, "
            f"TV excess T {out['windows'][name]['TV_excess_T']:.3f}")
    out["x"] = x[win].tolist()
    out["exact"] = {"rho": ex_rho.tolist(), "u": ex_u.tolist(), "T": ex_T.tolist()}
    out["profiles"] = {k: ({q: np.array(v[q])[win].tolist() for q in v} if v else None)
                       for k, v in res["profiles"].items()}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["laplace", "coexistence", "profile", "energy", "sod", "spurious", "droplet",
                                      "floor", "cooling"])
    ap.add_argument("--cap", type=int, default=1_000_000)
    ap.add_argument("--orders", default=None, help="window orders and scheme names (energy, spurious)")
    args = ap.parse_args()
    if args.study == "sod":
        print(json.dumps(sod()))
        return
    if args.orders and args.study in ("energy", "spurious"):
        fn = energy if args.study == "energy" else spurious
        print(json.dumps(fn(cap=args.cap, orders=V.parse_specs(args.orders))))
        return
    if args.study == "spurious":
        print(json.dumps(spurious(cap=args.cap)))
        return
    if args.study == "droplet":
        print(json.dumps(droplet_currents(cap=args.cap)))
        return
    if args.study == "floor":
        print(json.dumps(slab_floor(steps=args.cap)))
        return
    if args.study == "cooling":
        print(json.dumps(cooling(stage_steps=args.cap)))
        return
    fn = {"laplace": laplace, "coexistence": coexistence, "profile": profile, "energy": energy}[args.study]
    print(json.dumps(fn(cap=args.cap)))


if __name__ == "__main__":
    main()
