"""Writes sweep_64_oracle.json: the FP64 oracle's runs of the droplet sweep
(64 D2Q9 SRT droplets drawn by workload.sweep_items(64, seed=1906): sides
U{64..512}, R U{8..min(100, side/3)}, G U[-5.5, -4.5], tau U{0.8, 1.0, 1.2},
force-stencil order U{4, 6, 8, 10}, psi = 1 - exp(-rho), the seeded tanh
start; the droplet test of Sec. 3 repeated over a parameter sweep).

Stored:
  early   every item after `early_steps` (2,000) steps: the observables and
          the density and velocity along the x line through the centre;
  steady  the `n_steady` (4) items with the smallest grids, run until the
          steady-state rule holds: max|u| checked every 100 steps and the run
          stopped at the first check whose change from the previous check is
          below 1e-10 (the literal rule, FP64).  The step it stopped at, the
          observables and the centre lines there;
  tails   for each steady item that converges, the same oracle run sampled
          every `tail_every` (500) steps up to `tail_steps` (200,000): the
          observables at each sample.  The literal rule can fire at a turning
          point of max|u| while the state still relaxes, so a run that stops
          elsewhere is compared with the oracle's state at its own step.

Only the oracle computes these values.  The stored file came from
    python tests/golden/make_sweep_64_oracle.py
(each item in its own single-threaded process, -j of them at a time; about
25 min with -j 2), and the tails were added to it by
    python tests/golden/make_sweep_64_oracle.py --tails-only -j 3
(about 20 min).
"""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sweep_64_oracle.json")
SEED, N_ITEMS = 1906, 64


def _plain(ob):
    return {k: (float(v) if np.ndim(v) == 0 else [float(x) for x in v]) for k, v in ob.items()}


def _record(o, fl):
    from oracle import oracle as O
    ob = _plain(O.observables(fl, o.cs2, o.G, o.c0))
    c = [s // 2 for s in o.shape]
    return {"step": o.steps, "obs": ob, "rho_line": fl["rho"][:, c[1]].tolist(),
            "u_line": [fl["u"][d][:, c[1]].tolist() for d in range(2)]}


def _oracle(k):
    from oracle import oracle as O
    from workload import droplet_rho, sweep_items
    it = sweep_items(N_ITEMS, seed=SEED)[k]
    rho0 = droplet_rho((it["side"],) * 2, it["R"], seed=it["seed"])
    return O.Oracle(rho0, "D2Q9", order=it["order"], G=it["G"], tau=it["tau"])


def run_early(k, steps):
    t0 = time.time()
    o = _oracle(k).step(steps)
    r = _record(o, o.fields())
    r["item"], r["seconds"] = k, time.time() - t0
    return r


def run_steady(k, tol, every, max_steps):
    t0 = time.time()
    o = _oracle(k)
    prev = None
    while o.steps < max_steps:
        o.step(every)
        fl = o.fields()
        mu = float(np.sqrt((fl["u"] ** 2).sum(axis=0)).max())
        if prev is not None and abs(mu - prev) < tol:
            r = _record(o, fl)
            r.update(item=k, converged=True, seconds=time.time() - t0)
            return r
        prev = mu
    r = _record(o, o.fields())
    r.update(item=k, converged=False, seconds=time.time() - t0)
    return r


def run_tail(k, every, steps):
    from oracle import oracle as O
    t0 = time.time()
    o = _oracle(k)
    at, obs = [], {}
    while o.steps < steps:
        o.step(every)
        fl = o.fields()
        ob = _plain(O.observables(fl, o.cs2, o.G, o.c0))
        at.append(o.steps)
        for key in ("max_u", "mean_u", "l2_u", "dp", "rho_min", "rho_max", "mass"):
            obs.setdefault(key, []).append(ob[key])
    return {"item": k, "every": every, "steps": at, "obs": obs, "seconds": time.time() - t0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=2)
    ap.add_argument("--early-steps", type=int, default=2000)
    ap.add_argument("--n-steady", type=int, default=4)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--max-steps", type=int, default=400000)
    ap.add_argument("--items", type=int, default=N_ITEMS, help="first N items only (for a quick check)")
    ap.add_argument("--out", default=OUT)
    ap.add_argument("--tail-every", type=int, default=500)
    ap.add_argument("--tail-steps", type=int, default=200000)
    ap.add_argument("--tails-only", action="store_true",
                    help="add the tails of the converged steady items to the existing file")
    a = ap.parse_args()
    os.environ["OMP_NUM_THREADS"] = "1"   # one core per item; set before any worker loads the oracle
    if a.tails_only:
        with open(a.out) as fh:
            res = json.load(fh)
        ks = [s["item"] for s in res["steady"] if s["converged"]]
        t0 = time.time()
        with ProcessPoolExecutor(max_workers=a.j) as ex:
            fs = {ex.submit(run_tail, k, a.tail_every, a.tail_steps): k for k in ks}
            tails = []
            for f in fs:
                r = f.result()
                tails.append(r)
                print("tail item %d: %d samples, %.0f s (total %.0f s)" % (
                    r["item"], len(r["steps"]), r["seconds"], time.time() - t0), flush=True)
        res["tail_every"], res["tail_steps"] = a.tail_every, a.tail_steps
        res["tails"] = sorted(tails, key=lambda r: r["item"])
        with open(a.out, "w") as fh:
            json.dump(res, fh)
        print("wrote", a.out, flush=True)
        return
    from workload import sweep_items
    its = sweep_items(N_ITEMS, seed=SEED)
    smallest = sorted(range(N_ITEMS), key=lambda i: (its[i]["side"], i))[:a.n_steady]
    order = sorted(range(a.items), key=lambda i: -its[i]["side"])   # largest first: better packing
    t0 = time.time()
    early, steady = {}, {}
    with ProcessPoolExecutor(max_workers=a.j) as ex:
        fs = {ex.submit(run_steady, k, a.tol, a.every, a.max_steps): ("steady", k) for k in smallest}
        fs.update({ex.submit(run_early, k, a.early_steps): ("early", k) for k in order})
        for f in fs:
            kind, k = fs[f]
            r = f.result()
            (early if kind == "early" else steady)[k] = r
            print("%s item %d (side %d, E%d): step %d, max|u| %.6e, %.0f s (total %.0f s)" % (
                kind, k, its[k]["side"], its[k]["order"], r["step"], r["obs"]["max_u"], r["seconds"],
                time.time() - t0), flush=True)
    res = {"seed": SEED, "n_items": N_ITEMS, "items": its, "early_steps": a.early_steps,
           "tol": a.tol, "every": a.every, "max_steps": a.max_steps,
           "early": [early[k] for k in sorted(early)], "steady": [steady[k] for k in smallest],
           "oracle_seconds": time.time() - t0}
    with open(a.out, "w") as fh:
        json.dump(res, fh)
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    main()
