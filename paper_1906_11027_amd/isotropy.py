"""Spurious currents of a static droplet versus the isotropy order of the
interaction force (Sec. 2 and 3: E4, E6, E8, E10 force stencils), on the
D2Q9 SRT model with psi = 1 - exp(-rho), G = -5, tau = 1, at 256^2 with a
droplet of radius 40, in the FP64 state and in the FP32 state with the
automatic storage shift (the median initial density: the vapour) and with
the shift 1.

Each run takes a fixed number of steps (no stopping rule) and records the
FP64 observables -- max, mean and RMS |u| over the field, the Laplace
pressure jump between the droplet centre and the corner, the density
extremes and the mass -- every `every` steps.  The FP32 and FP64 fields
at the end are compared node by node, over the field and over the vapour
(rho < 0.3).

Two companion runs of the same droplet test:
    --case d3q19   the D3Q19 MRT droplet, 128^3 periodic, E4/E6/E8 3D force,
                   R = 24, G = -5, tau = 1 (MRT rates 1.2), 20,000 steps,
                   FP64 and FP32 with either shift;
    --case small   the 64^2 D2Q9 E4 droplet, R = 16, FP64 state, 10,000
                   steps: spurious max|u| and the Laplace jump.

Usage: python -m paper_1906_11027_amd.isotropy [--case orders|d3q19|small] [--steps N] [--every K] [--out FILE]
"""
import argparse
import json
import time

import numpy as np

from .sc_lbm import Sim

ORDERS = (4, 6, 8, 10)
KEYS = ("max_u", "mean_u", "l2_u", "dp", "rho_in", "rho_out", "rho_min", "rho_max", "radius", "mass")


def droplet(shape=(256, 256), R=40, seed=2):
    from workload import droplet_rho
    return droplet_rho(shape, R, seed=seed)


def run_one(rho0, order, precision, steps, every, G=-5.0, tau=1.0, rho_ref="auto", lattice="D2Q9", **kw):
    import torch
    if every < 1 or steps % every:
        raise ValueError("steps (%d) must be a multiple of every (%d)" % (steps, every))
    sim = Sim(rho0, lattice, order=order, G=G, tau=tau, precision=precision, obs_every=every, rho_ref=rho_ref,
              **kw)
    shift = sim.rho_ref
    traj = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc = 0
    for _ in range(steps // every):
        rc, _ = sim.step(every)
        o = sim.observe(fields=False)["obs"]
        traj.append({"step": int(o["step"]), **{k: float(o[k]) for k in KEYS}})
        if rc != 0:
            break
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = sim.observe()
    sim.close()
    return {"order": order, "precision": precision, "rho_ref": shift, "rc": int(rc), "wall_s": wall, "traj": traj,
            "final": traj[-1] if traj else None}, out["rho"], out["u"]


RUNS = (("fp64", "auto"), ("fp32", "auto"), ("fp32", 1.0))


def run(steps=50000, every=5000, shape=(256, 256), R=40, seed=2, log=print):
    rho0 = droplet(shape, R, seed)
    res = {"shape": list(shape), "R": R, "seed": seed, "G": -5.0, "tau": 1.0, "steps": steps, "every": every,
           "runs": [], "fp32_vs_fp64": {}}
    fields = {}
    for order in ORDERS:
        for prec, shift in RUNS:
            r, rho, u = run_one(rho0, order, prec, steps, every, rho_ref=shift)
            res["runs"].append(r)
            fields[(order, prec, r["rho_ref"])] = (rho, u)
            f = r["final"]
            log("E%d %s shift %.4f: %d steps in %.2f s, max|u| %.4e mean|u| %.4e dp %.6e" % (
                order, prec, r["rho_ref"], f["step"], r["wall_s"], f["max_u"], f["mean_u"], f["dp"]))
        (r64, u64), = [v for k, v in fields.items() if k[0] == order and k[1] == "fp64"]
        vap = r64 < 0.3
        m64 = np.sqrt((u64 ** 2).sum(axis=0)).max()
        for (o, prec, shift), (r32, u32) in fields.items():
            if o != order or prec != "fp32":
                continue
            du = np.sqrt(((u32 - u64) ** 2).sum(axis=0))
            res["fp32_vs_fp64"]["E%d shift %.4f" % (order, shift)] = {
                "max_abs_rho": float(np.abs(r32 - r64).max()),
                "max_abs_u": float(du.max()),
                "max_abs_u_rel_to_max_u": float(du.max() / m64),
                "vapour_median_abs_u": float(np.median(du[vap])),
            }
    return res, fields


def _compare(fields, ref_key, vapour):
    (r64, u64) = fields[ref_key]
    m64 = np.sqrt((u64 ** 2).sum(axis=0)).max()
    vap = r64 < vapour
    out = {}
    for key, (r32, u32) in fields.items():
        if key == ref_key:
            continue
        du = np.sqrt(((u32 - u64) ** 2).sum(axis=0))
        out["%s shift %.4f" % key] = {"max_abs_rho": float(np.abs(r32 - r64).max()), "max_abs_u": float(du.max()),
                                      "max_abs_u_rel_to_max_u": float(du.max() / m64),
                                      "vapour_median_abs_u": float(np.median(du[vap]))}
    return out


def run_d3q19(steps=20000, every=2000, log=print, orders=(4, 6, 8)):
    """The D3Q19 MRT droplet: 128^3, R = 24, the 3D force stencils E4, E6,
    E8, FP64 and FP32 with either shift."""
    from workload import droplet_rho
    rho0 = droplet_rho((128, 128, 128), 24, seed=3)
    res = {"lattice": "D3Q19", "collision": "mrt", "shape": [128] * 3, "R": 24, "seed": 3, "G": -5.0, "tau": 1.0,
           "orders": list(orders), "steps": steps, "every": every, "runs": [], "fp32_vs_fp64": {}}
    out = {}
    for order in orders:
        fields = {}
        for prec, shift in RUNS:
            r, rho, u = run_one(rho0, order, prec, steps, every, rho_ref=shift, lattice="D3Q19", collision="mrt")
            res["runs"].append(r)
            fields[(prec, r["rho_ref"])] = (rho, u)
            f = r["final"]
            log("D3Q19 MRT E%d %s shift %.4f: %d steps in %.2f s, max|u| %.4e mean|u| %.4e dp %.6e" % (
                order, prec, r["rho_ref"], f["step"], r["wall_s"], f["max_u"], f["mean_u"], f["dp"]))
        ref = [k for k in fields if k[0] == "fp64"][0]
        for key, v in _compare(fields, ref, 0.3).items():
            res["fp32_vs_fp64"]["E%d %s" % (order, key)] = v
        out.update({("E%d" % order,) + k: v for k, v in fields.items()})
    return res, out


def run_small(steps=10000, every=1000, log=print):
    """The 64^2 D2Q9 E4 droplet (R = 16) in the FP64 state."""
    rho0 = droplet((64, 64), 16, 1)
    r, rho, u = run_one(rho0, 4, "fp64", steps, every)
    f = r["final"]
    log("64^2 E4 FP64: %d steps in %.2f s, max|u| %.6e dp %.9e" % (f["step"], r["wall_s"], f["max_u"], f["dp"]))
    return {"lattice": "D2Q9", "shape": [64, 64], "R": 16, "seed": 1, "G": -5.0, "tau": 1.0, "order": 4,
            "steps": steps, "every": every, "runs": [r]}, {(4, "fp64", r["rho_ref"]): (rho, u)}


def main(argv=None):
    ap = argparse.ArgumentParser(description="spurious currents vs force isotropy order, 256^2 droplet")
    ap.add_argument("--case", choices=("orders", "d3q19", "small"), default="orders")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--every", type=int, default=None)
    ap.add_argument("--out", default=None)
    ap.add_argument("--fields", default=None, help="write the final fields to this .npz")
    a = ap.parse_args(argv)
    fn, steps, every = {"orders": (run, 50000, 5000), "d3q19": (run_d3q19, 20000, 2000),
                        "small": (run_small, 10000, 1000)}[a.case]
    res, fields = fn(a.steps or steps, a.every or every, log=lambda m: print(m, flush=True))
    print(json.dumps({k: v for k, v in res.items() if k != "runs"}), flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(res, fh, indent=1)
    if a.fields:
        np.savez(a.fields, **{"%s_e%s_%s_%.4f" % (q, str(o).lstrip("E"), p, sh): v
                              for (o, p, sh), fv in fields.items() for q, v in zip(("rho", "u"), fv)})
    return res


if __name__ == "__main__":
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main()
