"""Writes droplet_128_d3q19_oracle.json: the FP64 oracle's run of the 3D
droplet (D3Q19 MRT, stress moments at 1/tau = 1, other non-conserved
moments at 1.2; E8 3D force, psi = 1 - exp(-rho), G = -5, 128^3 periodic,
spherical droplet R = 24 from the seeded tanh start; Sec. 2, 3).  Stored:
the observables every `every` steps and, at the end, the density and
velocity along the x line through the centre.

Only the oracle computes these values.  The stored file came from
    python tests/golden/make_droplet_128_d3q19.py
(2,000 steps; about 25 min on 8 cores).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from workload import droplet_rho  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "droplet_128_d3q19_oracle.json")


def _plain(ob):
    return {k: (float(v) if np.ndim(v) == 0 else [float(x) for x in v]) for k, v in ob.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--every", type=int, default=500)
    a = ap.parse_args()
    shape, R, seed, G, tau, order = (128, 128, 128), 24, 3, -5.0, 1.0, 8
    t0 = time.time()
    o = O.Oracle(droplet_rho(shape, R, seed=seed), "D3Q19", order=order, G=G, tau=tau, collision="mrt")
    traj = []
    for _ in range(a.steps // a.every):
        o.step(a.every)
        fl = o.fields()
        ob = _plain(O.observables(fl, o.cs2, o.G, o.c0))
        ob["step"] = o.steps
        traj.append(ob)
        print("%d steps (%.0f s), max|u| %.6e" % (o.steps, time.time() - t0, ob["max_u"]), flush=True)
    c = [s // 2 for s in shape]
    res = {"lattice": "D3Q19", "collision": "mrt", "shape": list(shape), "R": R, "seed": seed, "G": G,
           "tau": tau, "order": order, "psi": "exp", "steps": a.steps, "every": a.every, "traj": traj,
           "oracle_seconds": time.time() - t0, "threads": O.num_threads(), "line_y": c[1], "line_z": c[2],
           "rho_line": fl["rho"][:, c[1], c[2]].tolist(),
           "u_line": [fl["u"][d][:, c[1], c[2]].tolist() for d in range(3)]}
    with open(OUT, "w") as fh:
        json.dump(res, fh, indent=1)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
