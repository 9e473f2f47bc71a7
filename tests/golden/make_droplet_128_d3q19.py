"""Writes droplet_128_d3q19_oracle.json: the FP64 oracle's run of the 3D
droplet (D3Q19 MRT, stress moments at 1/tau = 1, other non-conserved
moments at 1.2; E8 3D force, psi = 1 - exp(-rho), G = -5, 128^3 periodic,
spherical droplet R = 24 from the seeded tanh start; Sec. 2, 3) over the
configuration's full length of 20,000 steps.  Stored: the observables
every `every` steps, and the density and velocity along the x line
through the centre at 2,000 steps and at the end.

Only the oracle computes these values.  The stored file came from
    python tests/golden/make_droplet_128_d3q19.py
(20,000 steps; 5.8 h on 6 OpenMP threads).  The run saves the oracle's
distributions every `ckpt_every` steps to --ckpt (outside the repository)
and resumes from there when restarted: a step depends only on the
distributions, so a resumed run is bitwise the same as an uninterrupted one.
"""
import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from workload import droplet_rho  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "droplet_128_d3q19_oracle.json")
SHAPE, R, SEED, G, TAU, ORDER = (128, 128, 128), 24, 3, -5.0, 1.0, 8


def _plain(ob):
    return {k: (float(v) if np.ndim(v) == 0 else [float(x) for x in v]) for k, v in ob.items()}


def _lines(fl):
    c = [s // 2 for s in SHAPE]
    return fl["rho"][:, c[1], c[2]].tolist(), [fl["u"][d][:, c[1], c[2]].tolist() for d in range(3)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--every", type=int, default=500)
    ap.add_argument("--ckpt-every", type=int, default=2000)
    ap.add_argument("--early-line", type=int, default=2000, help="also store the centre line at this step")
    ap.add_argument("--out", default=OUT)
    ap.add_argument("--ckpt", default=os.path.join(tempfile.gettempdir(), "droplet_128_d3q19_oracle_ckpt.npz"))
    a = ap.parse_args()
    assert a.steps % a.every == 0 and a.ckpt_every % a.every == 0 and a.early_line % a.every == 0
    t0 = time.time()
    o = O.Oracle(droplet_rho(SHAPE, R, seed=SEED), "D3Q19", order=ORDER, G=G, tau=TAU, collision="mrt")
    traj, early, spent = [], None, 0.0
    if os.path.exists(a.ckpt):
        ck = np.load(a.ckpt)
        meta = json.loads(str(ck["meta"]))
        o.set_f(ck["f"])
        o.steps = int(meta["steps"])
        traj, early, spent = meta["traj"], meta["early"], float(meta["seconds"])
        print("resumed at %d steps from %s" % (o.steps, a.ckpt), flush=True)
    while o.steps < a.steps:
        o.step(a.every)
        fl = o.fields()
        ob = _plain(O.observables(fl, o.cs2, o.G, o.c0))
        ob["step"] = o.steps
        traj.append(ob)
        if o.steps == a.early_line:
            rl, ul = _lines(fl)
            early = {"step": o.steps, "rho_line": rl, "u_line": ul}
        print("%d steps (%.0f s), max|u| %.6e" % (o.steps, spent + time.time() - t0, ob["max_u"]), flush=True)
        if o.steps % a.ckpt_every == 0 and o.steps < a.steps:
            meta = {"steps": o.steps, "traj": traj, "early": early, "seconds": spent + time.time() - t0}
            tmp = a.ckpt + ".tmp.npz"
            np.savez(tmp, f=o.get_f(), meta=json.dumps(meta))
            os.replace(tmp, a.ckpt)
    fl = o.fields()
    rl, ul = _lines(fl)
    c = [s // 2 for s in SHAPE]
    res = {"lattice": "D3Q19", "collision": "mrt", "shape": list(SHAPE), "R": R, "seed": SEED, "G": G,
           "tau": TAU, "order": ORDER, "psi": "exp", "steps": a.steps, "every": a.every, "traj": traj,
           "oracle_seconds": spent + time.time() - t0, "threads": O.num_threads(), "line_y": c[1],
           "line_z": c[2], "rho_line": rl, "u_line": ul, "early": early}
    with open(a.out, "w") as fh:
        json.dump(res, fh, indent=1)
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    main()
