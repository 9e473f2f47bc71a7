"""The measurements of Sec. 3 run through the library: a droplet's spurious
currents versus reduced temperature, and the coexistence densities and
interface thickness of a flat interface, for the models the paper compares.

Models (name -> lattice, force-stencil order, tau):
    D2Q9-ISO4   D2Q9, E4, tau = 1        the standard model
    D2Q9-ISO6   D2Q9, E6, tau = 1        higher-order force only
    D2Q9-ISO8   D2Q9, E8, tau = 1        (Shan's improvement)
    D2Q13T      D2Q13, E6, tau = 1       same relaxation time
    D2Q13V      D2Q13, E6, tau = 11/12   same viscosity as D2Q9 at tau = 1
    D2Q25T      D2Q25, E8, tau = 1
    D2Q25V      D2Q25, E8, tau = 19/24
All use the Peng-Robinson pseudo-potential and the exact difference method
(Sec. 3).  With that psi the force does not depend on G or c0 (psi^2 scales
as 1 / (G c0)), so G = -1 and c0 = 1/3 are placeholders.

Droplet (Sec. 3): 60 x 60 periodic, r0 = 15 at the centre, tanh profile
between the Maxwell densities.  Flat interface: a liquid slab across a
periodic strip.  Wall droplet (Sec. 3, last experiment): a drop on the
bottom wall of a channel (walls two nodes thick, standard bounce-back) at
T = 0.9 Tc, wettability set by the virtual wall density rho_w.  Runs use
the FP64 state and stop when max |u| changes by less than `tol` between
checks.

Usage: python -m paper_1906_11027_amd.experiments [--droplet] [--flat] [--wall] [--out FILE]
"""
import argparse
import json
import sys

import numpy as np

from . import eos as P
from .sc_lbm import SC_E_NONFINITE, Sim

MODELS = {
    "D2Q9-ISO4": ("D2Q9", 4, 1.0),
    "D2Q9-ISO6": ("D2Q9", 6, 1.0),
    "D2Q9-ISO8": ("D2Q9", 8, 1.0),
    "D2Q13T": ("D2Q13", 6, 1.0),
    "D2Q13V": ("D2Q13", 6, 11.0 / 12.0),
    "D2Q25T": ("D2Q25", 8, 1.0),
    "D2Q25V": ("D2Q25", 8, 19.0 / 24.0),
}
TEMPERATURES = (0.6, 0.65, 0.7, 0.725, 0.75, 0.8, 0.85, 0.9, 0.95)


def tanh_profile(d, rho_l, rho_v, width):
    """Liquid where the signed distance d < 0."""
    return 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh(2.0 * d / width)


def droplet_init(shape, r0, rho_l, rho_v, width):
    x = np.arange(shape[0])[:, None] - shape[0] / 2.0
    y = np.arange(shape[1])[None, :] - shape[1] / 2.0
    return tanh_profile(np.sqrt(x * x + y * y) - r0, rho_l, rho_v, width)


def slab_init(n, ny, thickness, rho_l, rho_v, width):
    d = np.abs(np.arange(n) - n / 2.0) - thickness / 2.0
    return np.repeat(tanh_profile(d, rho_l, rho_v, width)[:, None], ny, axis=1)


def run_model(model, Tr, rho0, max_steps, tol, precision="fp64", obs_every=500, solid=None, rho_w=None):
    lattice, order, tau = MODELS[model]
    e = P.params_at(Tr)
    sim = Sim(rho0, lattice, order=order, tau=tau, G=-1.0, psi="pr", eos=e, forcing="edm",
              precision=precision, obs_every=obs_every)
    if solid is not None:
        sim.set_walls(solid, rho_w)
    rc, steps = sim.step(max_steps, tol=tol)
    out = sim.observe()
    sim.close()
    out["steps"] = steps
    out["diverged"] = rc == SC_E_NONFINITE or not np.all(np.isfinite(out["rho"]))
    out["converged"] = out["obs"]["converged_by"] > 0 or (not out["diverged"] and steps < max_steps)
    return out


def droplet(model, Tr, shape=(60, 60), r0=15.0, width=4.0, max_steps=400000, tol=1e-11):
    """Steady droplet: maximum and field-averaged spurious speed (Sec. 3)."""
    rv, rl = P.maxwell(P.params_at(Tr))
    r = run_model(model, Tr, droplet_init(shape, r0, rl, rv, width), max_steps, tol)
    o = r["obs"]
    return {"model": model, "Tr": Tr, "max_u": o["max_u"], "mean_u": o["mean_u"], "rho_in": o["rho_in"],
            "rho_out": o["rho_out"], "dp": o["dp"], "radius": o["radius"], "steps": r["steps"],
            "converged": bool(r["converged"]), "diverged": bool(r["diverged"]),
            "maxwell": [rv, rl]}


def interface_thickness(prof, rho_v, rho_l):
    """Width of the region 1.05 rho_v <= rho <= 0.95 rho_l across one
    interface of a monotone profile segment, with the two crossings placed
    by linear interpolation between nodes."""
    lo, hi = 1.05 * rho_v, 0.95 * rho_l

    def crossing(level):
        for i in range(len(prof) - 1):
            a, b = prof[i], prof[i + 1]
            if (a - level) * (b - level) <= 0 and a != b:
                return i + (level - a) / (b - a)
        return float("nan")
    return abs(crossing(hi) - crossing(lo))


def flat_interface(model, Tr, n=200, ny=4, thickness=100.0, width=4.0, max_steps=600000, tol=1e-12):
    """Coexistence densities (slab centre / far vapour) and the interface
    thickness (Sec. 3), from a steady liquid slab across a periodic strip."""
    rv, rl = P.maxwell(P.params_at(Tr))
    r = run_model(model, Tr, slab_init(n, ny, thickness, rl, rv, width), max_steps, tol)
    prof = r["rho"][:, 0]
    rho_l, rho_v = float(prof[n // 2]), float(prof[0])
    # left interface: from the vapour at x = 0 up to the liquid at the centre
    th = interface_thickness(prof[: n // 2 + 1], rho_v, rho_l)
    return {"model": model, "Tr": Tr, "rho_l": rho_l, "rho_v": rho_v, "thickness": th,
            "max_u": r["obs"]["max_u"], "steps": r["steps"], "converged": bool(r["converged"]),
            "diverged": bool(r["diverged"]), "maxwell": [rv, rl]}


def channel(shape, layers=2):
    """Solid mask: walls `layers` nodes thick at the bottom and top (y)."""
    m = np.zeros(shape, dtype=bool)
    m[:, :layers] = True
    m[:, shape[1] - layers:] = True
    return m


def _crossing(prof, level, start, step):
    """Fractional index where prof crosses `level` walking from `start`."""
    i = start
    while 0 <= i + step < len(prof):
        a, b = prof[i], prof[i + step]
        if (a - level) * (b - level) <= 0 and a != b:
            return i + step * (level - a) / (b - a)
        i += step
    return float("nan")


def contact_angle(rho, layers, rho_l, rho_v, skip=3):
    """Contact angle (degrees, through the liquid) of a drop on the bottom
    wall.  The mid-density contour is located on every row from `skip`
    nodes above the wall up (the rows next to the wall carry the wall's own
    adsorption layer), fitted with a circle by linear least squares, and
    intersected with the wall plane y_w (half-way between the last solid
    and the first fluid row): cos(theta) = (y_w - y_c) / R.  A drop whose
    fitted circle stays clear of the wall reads 180 degrees, liquid across
    the whole width 0.  Returns (theta, circle radius, centre height)."""
    mid = 0.5 * (rho_l + rho_v)
    yw = layers - 0.5
    ny = rho.shape[1]
    top_fluid = ny - layers
    if rho[:, layers + skip].min() > mid:
        return 0.0, float("inf"), float("nan")
    pts = []
    for y in range(layers + skip, top_fluid - skip):
        row = rho[:, y]
        if row.max() < mid or row.min() > mid:
            continue
        xc = int(np.argmax(row))
        for step in (-1, +1):
            xcr = _crossing(row, mid, xc, step)
            if np.isfinite(xcr):
                pts.append((xcr, float(y)))
    if len(pts) < 6:
        return 180.0, float("nan"), float("nan")
    P_ = np.array(pts)
    A = np.column_stack([P_[:, 0], P_[:, 1], np.ones(len(P_))])
    bvec = -(P_[:, 0] ** 2 + P_[:, 1] ** 2)
    (D, E, F), *_ = np.linalg.lstsq(A, bvec, rcond=None)
    xc0, yc0 = -D / 2.0, -E / 2.0
    R = float(np.sqrt(xc0 * xc0 + yc0 * yc0 - F))
    c = (yw - yc0) / R
    if c <= -1.0:
        return 180.0, R, float(yc0 - yw)
    return float(np.degrees(np.arccos(min(1.0, c)))), R, float(yc0 - yw)


def wall_droplet(model, rho_w, Tr=0.9, shape=(200, 100), r0=35.0, width=4.0, max_steps=400000, tol=1e-11):
    """Steady drop on a flat wall: contact angle and spurious speeds.  The
    wall nodes start at the vapour density: under full-way bounce-back the
    rest and wall-parallel populations of a solid node never leave it, so
    they should not carry the drop's liquid."""
    rv, rl = P.maxwell(P.params_at(Tr))
    x = np.arange(shape[0])[:, None] - shape[0] / 2.0
    y = np.arange(shape[1])[None, :] - 2.0
    rho0 = tanh_profile(np.sqrt(x * x + y * y) - r0, rl, rv, width)
    solid = channel(shape, 2)
    rho0[solid] = rv
    r = run_model(model, Tr, rho0, max_steps, tol, solid=solid, rho_w=rho_w)
    theta, R, hc = contact_angle(r["rho"], 2, rl, rv)
    o = r["obs"]
    return {"model": model, "Tr": Tr, "rho_w": rho_w, "theta_deg": theta, "cap_radius": R, "centre_height": hc,
            "max_u": o["max_u"], "mean_u": o["mean_u"], "steps": r["steps"], "converged": bool(r["converged"]),
            "diverged": bool(r["diverged"])}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--droplet", action="store_true")
    ap.add_argument("--flat", action="store_true")
    ap.add_argument("--wall", action="store_true")
    ap.add_argument("--wall-densities", default="1.5,2.0,2.5,3.0,3.5,4.0,4.5")
    ap.add_argument("--models", default=",".join(MODELS))
    ap.add_argument("--temps", default=",".join(str(t) for t in TEMPERATURES))
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    models = args.models.split(",")
    temps = [float(t) for t in args.temps.split(",")]
    res = {"droplet": [], "flat": [], "wall": []}
    if args.wall:
        for rw in [float(v) for v in args.wall_densities.split(",")]:
            for m in ("D2Q9-ISO4", "D2Q9-ISO8", "D2Q13T", "D2Q25T"):
                d = wall_droplet(m, rw)
                print("wall", json.dumps(d), flush=True)
                res["wall"].append(d)
    for Tr in temps:
        for m in models:
            if args.droplet:
                d = droplet(m, Tr)
                print("droplet", json.dumps(d), flush=True)
                res["droplet"].append(d)
            if args.flat:
                f = flat_interface(m, Tr)
                print("flat", json.dumps(f), flush=True)
                res["flat"].append(f)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(res, fh, indent=1)
    return res


if __name__ == "__main__":
    main()
    sys.exit(0)
