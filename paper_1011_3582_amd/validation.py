"""Physics runs of the FFT-LB step at the paper's equation-of-state constants (a = 9/8,
b = 1/3, so T_c = rho_c = 1), on the GPU through the library, and the measurements taken on
their fields.  The references they are compared with (Maxwell densities, the planar
equilibrium profile, the surface tension of Eq. (56)) are not computed here: the studies in
tests/physics_studies.py build the start fields from them and compare.

  relax(): batched runs until each residual stays below a tolerance (or a cap), with a
      monitor called on the fields after every chunk;
  pressure_jump(), equimolar_radius(), bulk_densities(): the Laplace-law pressure jump
      dP = P_in - P_out (Sec. 4.2), the droplet radius, the bulk densities of a slab;
  energy(): the variation of the total energy, Delta e_T(t) = e_T(t) - e_T(0) (Eq. (17)), in
      the 128 x 128 phase separation of Sec. 3.5 (rho = 1 + 1e-3 noise, T = 0.85) for the
      windows k1..k4 and the exact wavenumber (Sec. 3.6, Fig. 8's comparison);
  triangle(): an equilateral triangular droplet with a sharp interface relaxes to a circle
      (Sec. 4.2); the largest speed u^s_max(t) for k1..k4 (Fig. 19's comparison);
  sod(): the modified Sod shock tube of the ideal-gas special case (a = b = K = q = 0, so the
      force term vanishes: the Watari-Tsutahara model), with the exact wavenumber and k1..k4
      (Sec. 3.6, Figs. 6-7), on a periodic grid holding the tube and its mirror image.

Run as `python -m paper_1011_3582_amd.validation energy|triangle|sod`; each prints one JSON line.
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


def droplet_from_profile(n, radius, profile, T, dx):
    """A droplet of the given radius (grid units) centred on the grid: rho(r) =
    profile((radius - r) dx), a function of the signed distance from the interface (positive
    inside), u = 0, uniform temperature T.  Returns (rho, ux, uy, T)."""
    r = _periodic_radius(n, n / 2.0, n / 2.0)
    rho = profile((radius - r) * dx)
    z = np.zeros_like(rho)
    return rho, z, z, np.full_like(rho, T)


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


def window_name(m):
    """Name of a derivative order: exact, k1..k4, CD (the central difference, order 5), NPS
    (the nine-point stencils, order 6)."""
    return {0: "exact", 5: "CD", 6: "NPS"}.get(m, f"k{m}")


# Discretisations of the comparisons by name: (derivative order, convection scheme), with the
# paper's legend 'convection' + 'force' for the finite-difference schemes of Sec. 3.1.
SCHEMES = {"CD+CD": (5, F.CONV_SPECTRAL), "LW+CD": (5, F.CONV_LW), "MLW1+CD": (5, F.CONV_MLW1),
           "MLW2+CD": (5, F.CONV_MLW2), "FL+CD": (5, F.CONV_FL), "NPS+NPS": (6, F.CONV_SPECTRAL)}


def scheme(spec):
    """(derivative order, convection scheme) of a window order (int) or a SCHEMES name."""
    return (int(spec), F.CONV_SPECTRAL) if isinstance(spec, (int, np.integer)) else SCHEMES[spec]


def scheme_name(spec):
    return window_name(int(spec)) if isinstance(spec, (int, np.integer)) else spec


def parse_specs(text):
    """Comma-separated window orders and scheme names, e.g. "4,CD+CD,LW+CD,NPS+NPS"."""
    return tuple(int(v) if v.strip().isdigit() else v.strip() for v in text.split(","))


def _chunked(b, n_inst, cap, every, record):
    """Advance a batch (nothing retires: tolerance 0) in chunks of `every` steps up to cap,
    calling record(steps) after each chunk; instances that go non-finite stop advancing."""
    done = 0
    record(0)
    while done < cap:
        n = min(every, cap - done)
        b.run(tol=0.0, consecutive=3, poll_every=min(n, 1000), max_steps=n, allow_unstable=True)
        done += n
        record(done)


def energy(n=128, orders=(1, 2, 3, 4, 0), cap=200_000, every=2000, seed=0, dt=1e-5, keep_fields=False):
    """Delta e_T(t) of the phase separation of Sec. 3.5 (a = 9/8, b = 1/3, T = 0.85,
    rho = 1 + 1e-3 U[-1, 1], seeded) for each window order (0 = exact wavenumber), each run
    measuring e_T with its own windowed gradient.  keep_fields: also return the initial fields
    and every run's final (rho, ux, uy, T) as numpy arrays (under "fields", not JSON)."""
    rng = np.random.default_rng(seed)
    rho = (1.0 + 1e-3 * rng.uniform(-1.0, 1.0, (n, n))).astype(np.float32)
    z = np.zeros_like(rho)
    T = np.full_like(rho, 0.85)
    params = [F.Params(a=A_PAPER, b=B_PAPER, m=scheme(m)[0], convection=scheme(m)[1], dt=dt, precision=1)
              for m in orders]
    b = F.Batch([_tensors(rho, z, z, T) for _ in orders], params)
    area = n * n * params[0].dx * params[0].dy
    series = {m: [] for m in orders}
    t0 = time.perf_counter()
    e0 = {}

    def record(steps):
        for i, m in enumerate(orders):
            try:
                g = b.instance(i).poll()
            except F.FFTLBError:
                series[m].append({"t": steps * params[i].dt, "de_T": None})
                continue
            e = g["energy"] / area                    # mean e_T over the domain
            e0.setdefault(m, e)
            series[m].append({"t": steps * params[i].dt, "de_T": e - e0[m], "umax": g["umax"]})
        if steps % (10 * every) == 0:
            log(f"energy {time.perf_counter() - t0:.0f} s, {steps} steps: " + ", ".join(
                f"{scheme_name(m)}: {series[m][-1]['de_T']}" for m in orders))

    _chunked(b, len(orders), cap, every, record)
    kept = None
    if keep_fields:
        kept = {"initial": tuple(a.astype(np.float64) for a in (rho, z, z, T))}
        for i, m in enumerate(orders):
            outs, _ = b.instance(i).moments(globals_=False)
            kept[scheme_name(m)] = tuple(o.cpu().numpy().astype(np.float64) for o in outs)
    b.close()
    final = {scheme_name(m): series[m][-1]["de_T"] for m in orders}
    return {"n": n, "T": 0.85, "a": A_PAPER, "b": B_PAPER, "noise": 1e-3, "seed": seed, "steps": cap, "dt": dt,
            "e_T0": e0, "final_de_T": final,
            "series": {(scheme_name(m)): series[m] for m in orders},
            **({"fields": kept} if keep_fields else {})}


def triangle(n=128, side=64.0, orders=(1, 2, 3, 4), cap=3_000_000, every=20_000, precision=1):
    """An equilateral triangle of side `side` grid units (centroid at the centre, one edge
    parallel to x), rho = 1.46 inside and 0.58 outside with a sharp interface, u = 0, T = 0.95,
    K = 1e-5 (Sec. 4.2); the largest speed against time for each window order."""
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    h = side * math.sqrt(3.0) / 2.0
    cx, cy = n / 2.0, n / 2.0
    yb = cy - h / 3.0                          # base edge; apex at cy + 2h/3
    inside = (y >= yb) & (np.abs(x - cx) <= (cy + 2.0 * h / 3.0 - y) / math.sqrt(3.0))
    rho = np.where(inside, 1.46, 0.58)
    z = np.zeros_like(rho)
    T = np.full_like(rho, 0.95)
    params = [F.Params(a=A_PAPER, b=B_PAPER, K=1e-5, m=scheme(m)[0], convection=scheme(m)[1], precision=precision)
              for m in orders]
    b = F.Batch([_tensors(rho, z, z, T) for _ in orders], params)
    series = {m: [] for m in orders}
    t0 = time.perf_counter()

    def record(steps):
        for i, m in enumerate(orders):
            try:
                g = b.instance(i).poll()
                series[m].append({"t": steps * params[i].dt, "umax": g["umax"], "residual": g["residual"]})
            except F.FFTLBError:
                series[m].append({"t": steps * params[i].dt, "umax": None, "residual": None})
        if steps % (10 * every) == 0:
            log(f"triangle {time.perf_counter() - t0:.0f} s, {steps} steps: " + ", ".join(
                f"{scheme_name(m)}: {series[m][-1]['umax']}" for m in orders))

    _chunked(b, len(orders), cap, every, record)
    shapes = {}
    for i, m in enumerate(orders):
        (r, _, _, _), _ = b.instance(i).moments(globals_=False)
        r = r.cpu().numpy().astype(np.float64)
        rr = _periodic_radius(n, cx, cy)
        mid = 0.5 * (1.46 + 0.58)
        ring = np.abs(r - mid) < 0.15
        shapes[scheme_name(m)] = {"radius_mean": float(rr[ring].mean()), "radius_std": float(rr[ring].std())}
    b.close()
    return {"n": n, "side": side, "T": 0.95, "K": 1e-5, "precision": precision, "steps": cap,
            "final_umax": {scheme_name(m): series[m][-1]["umax"] for m in orders}, "shape": shapes,
            "series": {scheme_name(m): series[m] for m in orders}}


def sod(nx=768, ny=4, orders=(0, 1, 2, 3, 4), steps=20_000, every=2000):
    """The modified Sod tube (Sec. 3.6): (rho, u, T) = (1, 0, 1) for x <= 0 and (0.125, 0, 0.5)
    for x > 0, dx = dy = 2.5e-3, dt = 1e-5, tau = 3e-4, a = b = K = q = 0, to t = 0.2.  The
    periodic grid holds the tube (cell centres x_i = (i - nx/2 + 1/2) dx) and, across its ends,
    the mirror problem; at t = 0.2 their waves have not met (|x| < 0.6 of the 0.96 half-width
    is the tube's own solution).  Returns x and the row-averaged rho, u_x, T at t = 0.2 of every
    window (None where the run became non-finite) and the largest speed over time."""
    dx = 2.5e-3
    x = (np.arange(nx) - nx / 2 + 0.5) * dx
    left = x <= 0.0
    rho = np.broadcast_to(np.where(left, 1.0, 0.125)[None, :], (ny, nx)).copy()
    T = np.broadcast_to(np.where(left, 1.0, 0.5)[None, :], (ny, nx)).copy()
    z = np.zeros_like(rho)
    params = [F.Params(dx=dx, dy=dx, dt=1e-5, tau=3e-4, K=0.0, H=0.0, zeta=0.0, q=0.0, a=0.0, b=0.0, m=m)
              for m in orders]
    b = F.Batch([_tensors(rho, z, z, T) for _ in orders], params)
    umax = {m: [] for m in orders}

    def record(n):
        for i, m in enumerate(orders):
            try:
                umax[m].append((n * 1e-5, b.instance(i).poll()["umax"]))
            except F.FFTLBError:
                umax[m].append((n * 1e-5, None))

    _chunked(b, len(orders), steps, every, record)
    prof = {}
    for i, m in enumerate(orders):
        name = window_name(m)
        try:
            b.instance(i).poll()
        except F.FFTLBError:
            prof[name] = None
            continue
        (r, ux, _, t), _ = b.instance(i).moments(globals_=False)
        prof[name] = {"rho": r.cpu().numpy().astype(np.float64).mean(axis=0).tolist(),
                      "u": ux.cpu().numpy().astype(np.float64).mean(axis=0).tolist(),
                      "T": t.cpu().numpy().astype(np.float64).mean(axis=0).tolist()}
    b.close()
    return {"nx": nx, "dx": dx, "t": steps * 1e-5, "x": x.tolist(), "profiles": prof,
            "umax": {(window_name(m)): v for m, v in umax.items()}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["energy", "triangle", "sod"])
    ap.add_argument("--cap", type=int, default=1_000_000)
    ap.add_argument("--dt", type=float, default=1e-5, help="time step of the energy study")
    ap.add_argument("--orders", default=None,
                    help="window orders (0: exact k) and scheme names (CD+CD, LW+CD, MLW1+CD, MLW2+CD, NPS+NPS)")
    args = ap.parse_args()
    if args.study == "energy":
        out = energy(cap=args.cap, dt=args.dt, orders=parse_specs(args.orders or "1,2,3,4,0"),
                     every=max(1000, int(round(2000 * 1e-5 / args.dt))))
    elif args.study == "sod":
        out = sod()
    else:
        out = triangle(cap=args.cap, orders=parse_specs(args.orders or "1,2,3,4"))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
