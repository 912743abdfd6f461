"""Physics validation of the FFT-LB step at the paper's equation-of-state constants
(a = 9/8, b = 1/3, so T_c = rho_c = 1), run on the GPU through the library.

  laplace(): droplets of several radii at T = 0.95 for K = 1e-5, 7.5e-6, 5e-6 relax in one
      batch; the pressure jump dP = P_in - P_out (P_in the mean bulk pressure over the sites
      within R/2 of the centre, P_out over those beyond 3R/2, Sec. 4.2) against 1/R gives the
      surface tension as the slope (Laplace law, Eq. (55)), compared with
      sigma = K int (d rho/dz)^2 dz of the planar equilibrium interface (Eq. (56)).
  profile(): a relaxed planar slab against the equilibrium profile of the square-gradient
      model (the interface integral of Eqs. (51)-(53)).
  coexistence(): slabs started with the densities of a temperature 0.02 T_c higher than
      their own relax to the coexistence curve of the Maxwell construction (Sec. 4.1,
      the temperature steps of the coexistence-curve study).

The relaxed fields come from the FFT-LB run alone; the references (Maxwell densities,
planar profile, surface tension) come from the van der Waals free energy.  Radii are the
equimolar radii of the relaxed droplets.  Run as `python -m paper_1011_3582_amd.validation
<study>`; each study prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import fftlb as F

A_PAPER, B_PAPER = 9.0 / 8.0, 1.0 / 3.0


def log(msg):
    print(f"[validation] {msg}", file=sys.stderr, flush=True)


def _tensors(*arrays):
    return tuple(torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)) for a in arrays)


def _periodic_radius(n, cx, cy):
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    dx = np.abs(x - cx)
    dy = np.abs(y - cy)
    return np.hypot(np.minimum(dx, n - dx), np.minimum(dy, n - dy))


def droplet_start(n, radius, T, K, dx, thermo):
    """A droplet of the given radius (grid units) with the planar equilibrium profile across
    its interface (liquid inside), at uniform temperature T."""
    r = _periodic_radius(n, n / 2.0, n / 2.0)
    rho = thermo.planar_profile((radius - r) * dx, T, A_PAPER, B_PAPER, K)
    z = np.zeros_like(rho)
    return rho, z, z, np.full_like(rho, T)


def _fields(b, n):
    out = []
    for i in range(n):
        (rho, _, _, T), _ = b.instance(i).moments(globals_=False)
        out.append((rho.cpu().numpy().astype(np.float64), T.cpu().numpy().astype(np.float64)))
    return out


def relax(fields, params, tol, cap, chunk=50000, label="", monitor=None):
    """Run instances in one batch until each residual stays below tol (3 polls) or cap steps;
    returns the status and the (rho, T) fields.  monitor(steps, fields) is called after every
    chunk (a convergence record of the study's own measurement)."""
    b = F.Batch([_tensors(*f) for f in fields], params)
    b.autotune(reps=3)
    t0 = time.perf_counter()
    done = 0
    while done < cap:
        n = min(chunk, cap - done)
        b.run(tol=tol, consecutive=3, poll_every=100, max_steps=n)
        done += n
        st = b.status()
        log(f"{label} {time.perf_counter() - t0:.0f} s, {done} steps: {int((st['state'] != 0).sum())}/{len(fields)} "
            f"retired, max residual {st['residual'].max():.2e}")
        if monitor is not None:
            monitor(done, _fields(b, len(fields)))
        if (st["state"] != 0).all():
            break
    st = b.status()
    out = _fields(b, len(fields))
    b.close()
    return st, out


def pressure_jump(rho, T, radius):
    """dP = P_in - P_out of Sec. 4.2 around the grid centre (radius in grid units)."""
    n = rho.shape[0]
    r = _periodic_radius(n, n / 2.0, n / 2.0)
    P = rho * T / (1.0 - B_PAPER * rho) - A_PAPER * rho * rho
    return float(P[r < 0.5 * radius].mean() - P[r > 1.5 * radius].mean())


def equimolar_radius(rho):
    """Radius (grid units) of the disc whose sharp-interface mass equals the droplet's excess:
    R^2 pi (rho_in - rho_out) = sum (rho - rho_out), rho_in / rho_out the centre / corner means."""
    n = rho.shape[0]
    r = _periodic_radius(n, n / 2.0, n / 2.0)
    rho_in = rho[r < 3].mean()
    rho_out = rho[r > 0.45 * n].mean()
    return math.sqrt((rho - rho_out).sum() / (math.pi * (rho_in - rho_out)))


def laplace(n=192, radii=(24, 28, 32, 36, 40), Ks=(1e-5, 7.5e-6, 5e-6), t_ratio=0.95, tol=1e-9, cap=1_000_000):
    from oracle import thermo  # references from the van der Waals free energy
    T = t_ratio * 8 * A_PAPER / (27 * B_PAPER)
    fields, params, keys = [], [], []
    for K in Ks:
        p = F.Params(a=A_PAPER, b=B_PAPER, K=K, precision=1)
        for R in radii:
            fields.append(droplet_start(n, R, T, K, p.dx, thermo))
            params.append(p)
            keys.append((K, R))
    dx = F.Params().dx
    history = []

    def fits(relaxed):
        out = {}
        for K in Ks:
            sel = [i for i, (k, _) in enumerate(keys) if k == K]
            inv_r = [1.0 / (equimolar_radius(relaxed[i][0]) * dx) for i in sel]
            dps = [pressure_jump(relaxed[i][0], relaxed[i][1], equimolar_radius(relaxed[i][0])) for i in sel]
            out[K] = np.polyfit(inv_r, dps, 1)
        return out

    def monitor(steps, relaxed):
        f = fits(relaxed)
        history.append({"steps": steps, "sigma_fit": {f"{K:g}": float(f[K][0]) for K in Ks}})
        log("  sigma fits " + ", ".join(f"{K:g}: {f[K][0]:.4e}" for K in Ks))

    st, relaxed = relax(fields, params, tol, cap, label="laplace", monitor=monitor)
    res = {"n": n, "T/Tc": t_ratio, "tol": tol, "cap": cap, "history": history, "K": {}}
    for K in Ks:
        inv_r, dps, rows = [], [], []
        for (k, R0), (rho, Tf), steps, state, resid in zip(keys, relaxed, st["steps"], st["state"], st["residual"]):
            if k != K:
                continue
            Req = equimolar_radius(rho)
            dp = pressure_jump(rho, Tf, Req)
            inv_r.append(1.0 / (Req * dx))
            dps.append(dp)
            rows.append({"R0": R0, "R_equimolar": Req, "dP": dp, "T_mean": float(Tf.mean()), "steps": int(steps),
                         "state": int(state), "residual": float(resid)})
        slope, intercept = np.polyfit(inv_r, dps, 1)
        t_end = float(np.mean([r["T_mean"] for r in rows]))
        sigma = thermo.surface_tension(t_end, A_PAPER, B_PAPER, K)
        res["K"][f"{K:g}"] = {"sigma_fit": float(slope), "intercept": float(intercept), "sigma_theory": sigma,
                              "rel_err": abs(slope - sigma) / sigma, "T_end": t_end, "droplets": rows}
        log(f"K {K:g}: sigma fit {slope:.4e}, theory {sigma:.4e} (T {t_end:.5f}), intercept {intercept:.2e}")
    return res


def slab_start(nx, ny, rho_of_x, T):
    rho = np.broadcast_to(rho_of_x[None, :], (ny, nx)).copy()
    z = np.zeros_like(rho)
    return rho, z, z, np.full_like(rho, T)


def bulk_densities(rho):
    """Vapour and liquid bulk densities of a slab with interfaces at nx/4 and 3nx/4: means
    over 32 columns at the centre of each phase."""
    prof = rho.mean(axis=0)
    nx = prof.size
    return float(np.concatenate([prof[:16], prof[-16:]]).mean()), float(prof[nx // 2 - 16: nx // 2 + 16].mean())


def coexistence(temps=(0.80, 0.82, 0.84, 0.86, 0.88, 0.90, 0.92, 0.94, 0.96, 0.98), step=0.02, nx=256, ny=4,
                tol=1e-10, cap=1_000_000):
    """Slabs (liquid in nx/4 < x <= 3nx/4) at T, started from the coexistence densities of T + step
    (tanh interfaces of the equilibrium width at T + step): the bulk densities must move to
    the coexistence curve at the relaxed temperature."""
    from oracle import thermo
    t_c = 8 * A_PAPER / (27 * B_PAPER)
    fields, params = [], []
    x = np.arange(nx, dtype=np.float64)
    for tr in temps:
        p = F.Params(a=A_PAPER, b=B_PAPER, precision=1)
        hot = min(tr + step, 0.995) * t_c
        dist = np.minimum(x - nx / 4.0, 3.0 * nx / 4.0 - x) * p.dx
        fields.append(slab_start(nx, ny, thermo.planar_profile(dist, hot, A_PAPER, B_PAPER, p.K), tr * t_c))
        params.append(p)
    history = []

    def monitor(steps, relaxed):
        row = {"steps": steps, "gap_error": []}
        for (rho, T) in relaxed:
            rv, rl = bulk_densities(rho)
            mv, ml = thermo.maxwell(float(T.mean()), A_PAPER, B_PAPER)
            row["gap_error"].append(max(abs(rv - mv), abs(rl - ml)) / (ml - mv))
        history.append(row)
        log("  worst distance to the curve (of the gap): " + f"{max(row['gap_error']):.2e}")

    st, relaxed = relax(fields, params, tol, cap, label="coexistence", monitor=monitor)
    rows = []
    for tr, (rho, T), steps, state in zip(temps, relaxed, st["steps"], st["state"]):
        rv, rl = bulk_densities(rho)
        t_end = float(T.mean())
        mv, ml = thermo.maxwell(t_end, A_PAPER, B_PAPER)
        sv, sl = thermo.maxwell(min(tr + step, 0.995) * t_c, A_PAPER, B_PAPER)
        rows.append({"T/Tc": tr, "T_end": t_end, "rho_v": rv, "rho_l": rl, "maxwell_v": mv, "maxwell_l": ml,
                     "start_v": sv, "start_l": sl, "gap_error": max(abs(rv - mv), abs(rl - ml)) / (ml - mv),
                     "start_gap_error": max(abs(sv - mv), abs(sl - ml)) / (ml - mv), "steps": int(steps),
                     "state": int(state)})
    return {"nx": nx, "ny": ny, "step": step, "tol": tol, "cap": cap, "slabs": rows, "history": history}


def profile(t_ratio=0.95, K=1e-5, nx=256, ny=4, start_width=2.0, tol=1e-10, cap=400_000):
    """A slab started from the equilibrium profile stretched by start_width (a non-equilibrium
    interface) relaxes; the relaxed profile is compared with the equilibrium profile of the
    square-gradient model at the relaxed temperature, centred at the relaxed interface."""
    from oracle import thermo
    t_c = 8 * A_PAPER / (27 * B_PAPER)
    T = t_ratio * t_c
    p = F.Params(a=A_PAPER, b=B_PAPER, K=K, precision=1)
    x = np.arange(nx, dtype=np.float64)
    dist = np.minimum(x - nx / 4.0, 3.0 * nx / 4.0 - x) * p.dx
    start = thermo.planar_profile(dist / start_width, T, A_PAPER, B_PAPER, K)
    st, relaxed = relax([slab_start(nx, ny, start, T)], [p], tol, cap, label="profile")
    rho, Tf = relaxed[0]
    prof = rho.mean(axis=0)
    t_end = float(Tf.mean())
    mv, ml = thermo.maxwell(t_end, A_PAPER, B_PAPER)
    # interface positions: where the profile crosses the mid density (linear interpolation)
    mid = 0.5 * (prof[:nx // 2].min() + prof[nx // 4: 3 * nx // 4].max())
    i = int(np.argmax(prof[: nx // 2] > mid))
    x0 = i - 1 + (mid - prof[i - 1]) / (prof[i] - prof[i - 1])
    theory = thermo.planar_profile((x - x0) * p.dx, t_end, A_PAPER, B_PAPER, K)
    win = slice(int(x0) - 24, int(x0) + 25)
    err = np.abs(prof[win] - theory[win]).max() / (ml - mv)
    start_err = np.abs(start[win] - thermo.planar_profile((x[win] - nx / 4) * p.dx, T, A_PAPER, B_PAPER, K)).max()
    return {"T/Tc": t_ratio, "K": K, "nx": nx, "start_width_factor": start_width, "T_end": t_end,
            "interface_x": x0, "max_err_of_gap": float(err), "start_max_err_of_gap": float(start_err / (ml - mv)),
            "steps": int(st["steps"][0]), "state": int(st["state"][0]), "residual": float(st["residual"][0]),
            "profile": [float(v) for v in prof[win]], "theory": [float(v) for v in theory[win]]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["laplace", "coexistence", "profile"])
    ap.add_argument("--cap", type=int, default=1_000_000)
    args = ap.parse_args()
    if args.study == "laplace":
        out = laplace(cap=args.cap)
    elif args.study == "coexistence":
        out = coexistence(cap=args.cap)
    else:
        out = profile(cap=args.cap)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
