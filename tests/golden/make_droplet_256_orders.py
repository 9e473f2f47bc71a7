"""Writes droplet_256_orders_oracle.json: the FP64 oracle's run of the static
droplet of the isotropy study (D2Q9 SRT, psi = 1 - exp(-rho), G = -5,
tau = 1, 256^2 periodic, droplet R = 40 from the seeded tanh start) for
force-stencil orders among E4, E6, E8, E10 (Sec. 2, 3).  Stored per order:
the observables every `every` steps and, at the end, the density and
velocity along the row and the column through the droplet centre.  Orders
already in the file are kept, so the orders can be run at different
lengths.

Only the oracle computes these values.  The stored file came from
    python tests/golden/make_droplet_256_orders.py --orders 8
    python tests/golden/make_droplet_256_orders.py --orders 4,6,10
(50,000 steps each; about 4-8 min per order on 8 cores).
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "droplet_256_orders_oracle.json")


def _plain(ob):
    return {k: (float(v) if np.ndim(v) == 0 else [float(x) for x in v]) for k, v in ob.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--orders", default="4,6,8,10")
    ap.add_argument("--steps", type=int, default=50000)
    ap.add_argument("--every", type=int, default=5000)
    a = ap.parse_args()
    shape, R, seed, G, tau = (256, 256), 40, 2, -5.0, 1.0
    res = {"lattice": "D2Q9", "shape": list(shape), "R": R, "seed": seed, "G": G, "tau": tau, "psi": "exp",
           "orders": {}}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            res["orders"] = json.load(fh)["orders"]
    for order in [int(v) for v in a.orders.split(",")]:
        t0 = time.time()
        o = O.Oracle(droplet_rho(shape, R, seed=seed), "D2Q9", order=order, G=G, tau=tau)
        traj = []
        for _ in range(a.steps // a.every):
            o.step(a.every)
            fl = o.fields()
            ob = _plain(O.observables(fl, o.cs2, o.G, o.c0))
            ob["step"] = o.steps
            traj.append(ob)
            print("E%d: %d steps (%.0f s), max|u| %.6e" % (order, o.steps, time.time() - t0, ob["max_u"]),
                  flush=True)
        cx, cy = shape[0] // 2, shape[1] // 2
        res["orders"][str(order)] = {
            "steps": a.steps, "every": a.every,
            "traj": traj, "oracle_seconds": time.time() - t0, "threads": O.num_threads(),
            "row_y": cy, "col_x": cx,
            "rho_row": fl["rho"][:, cy].tolist(), "ux_row": fl["u"][0][:, cy].tolist(),
            "uy_row": fl["u"][1][:, cy].tolist(),
            "rho_col": fl["rho"][cx, :].tolist(), "ux_col": fl["u"][0][cx, :].tolist(),
            "uy_col": fl["u"][1][cx, :].tolist(),
        }
        with open(OUT, "w") as fh:
            json.dump(res, fh, indent=1)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
