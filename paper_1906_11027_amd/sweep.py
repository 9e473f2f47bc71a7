"""Time to steady state of the droplet sweep (batched sweeps are an addition
to the paper's method).

The sweep's droplets -- sides U{64..512}, R U{8..min(100, side/3)}, G
U[-5.5, -4.5], tau U{0.8, 1.0, 1.2}, stencil order U{4, 6, 8, 10}, the tanh
start with its seeded +-1e-3 jitter -- are run to the steady-state rule
(max|u| changing by less than `tol` between checks every K steps; an FP32
state also stops on its resolution floor) two ways on the same GPU:

    batched   one FP32 sweep, one launch per two steps over the active
              droplets' tiles (the batched tuner's shape), converged droplets
              leaving the work list; then the same batch widened to FP64
              (sc_lbm_batch_promote) and finished to the literal rule;
    per-drop  plain FP64 runs, one droplet after the other (each with its own
              graph-replayed step loop).

The steady observables of the two (max and mean |u|, Laplace jump, density
extremes) are compared on the droplets both runs bring to steady state
(those that evaporate to the uniform field at rest are counted apart).

Usage: python -m paper_1906_11027_amd.sweep [--items N] [--tol T] [--max-steps N] [--out FILE]
"""
import argparse
import json
import time

import numpy as np

from .sc_lbm import Batch, Sim, batch_autotune


def _items(n_items, seed):
    from workload import droplet_rho, sweep_items
    its = sweep_items(n_items, seed=seed)
    return its, [{"rho0": droplet_rho((it["side"],) * 2, it["R"], seed=it["seed"]), "order": it["order"],
                  "G": it["G"], "tau": it["tau"]} for it in its]


def run(n_items=64, tol=1e-10, max_steps=200000, obs_every=100, seed=1906, log=print):
    import torch
    its, items = _items(n_items, seed)
    nodes = [it["rho0"].size for it in items]
    shape, _ = batch_autotune(items, steps=64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt = Batch(items, obs_every=obs_every, variant=shape)
    bt.step(max_steps, tol=tol)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    b_steps, b_by = zip(*[bt.status(k) for k in range(n_items)])
    b_obs = [bt.observe(k, fields=False)["obs"] for k in range(n_items)]
    log("batched FP32 (%s): %.2f s, converged %d of %d" % (bt.variant, t_batch, sum(1 for v in b_by if v > 0),
                                                          n_items))
    bt.promote()
    bt.step(max_steps, tol=tol)
    torch.cuda.synchronize()
    t_promoted = time.perf_counter() - t0
    p_steps, p_by = zip(*[bt.status(k) for k in range(n_items)])
    p_obs = [bt.observe(k, fields=False)["obs"] for k in range(n_items)]
    bt.close()
    log("then FP64 to the literal rule: %.2f s in all, converged %d of %d" % (
        t_promoted, sum(1 for v in p_by if v == 1), n_items))
    f_steps, f_wall, f_rc, f_obs = [], [], [], []
    t0 = time.perf_counter()
    for k, it in enumerate(items):
        t1 = time.perf_counter()
        sim = Sim(it["rho0"], "D2Q9", order=it["order"], G=it["G"], tau=it["tau"], precision="fp64",
                  obs_every=obs_every)
        rc, done = sim.step(max_steps, tol=tol)
        f_obs.append(sim.observe(fields=False)["obs"])
        sim.close()
        torch.cuda.synchronize()
        f_steps.append(int(done))
        f_rc.append(int(rc))
        f_wall.append(time.perf_counter() - t1)
        log("FP64 droplet %d/%d: side %d, R %d, order %d: %d steps, %.2f s" % (
            k + 1, n_items, its[k]["side"], its[k]["R"], its[k]["order"], done, f_wall[-1]))
    t_fp64 = time.perf_counter() - t0
    f_conv = [s < max_steps and rc == 0 for s, rc in zip(f_steps, f_rc)]
    both = [k for k in range(n_items) if f_conv[k] and b_by[k] > 0]
    # a sub-critical droplet evaporates: its steady state is the uniform
    # field at rest, where |u| is round-off of either precision
    drops = [k for k in both if f_obs[k]["rho_max"] - f_obs[k]["rho_min"] > 0.5]

    def rel(obs, key, k):
        return abs(obs[k][key] - f_obs[k][key]) / max(abs(f_obs[k][key]), 1e-300)

    def agreement(obs, ks):
        return {key: {"median": float(np.median([rel(obs, key, k) for k in ks])) if ks else None,
                      "max": float(np.max([rel(obs, key, k) for k in ks])) if ks else None}
                for key in ("max_u", "mean_u", "dp", "rho_min", "rho_max")}
    agree = agreement(b_obs, drops)
    both_p = [k for k in range(n_items) if f_conv[k] and p_by[k] == 1]
    drops_p = [k for k in both_p if f_obs[k]["rho_max"] - f_obs[k]["rho_min"] > 0.5]
    return {
        "items": n_items, "tol": tol, "max_steps": max_steps, "obs_every": obs_every, "nodes_total": int(sum(nodes)),
        "batched_fp32": {"wall_s": t_batch, "steps_max": int(max(b_steps)), "steps_mean": float(np.mean(b_steps)),
                         "converged_tol": int(sum(1 for v in b_by if v == 1)),
                         "converged_floor": int(sum(1 for v in b_by if v == 2)),
                         "nonfinite": int(sum(1 for v in b_by if v < 0)),
                         "not_converged": int(sum(1 for v in b_by if v == 0))},
        "per_droplet_fp64": {"wall_s": t_fp64, "steps_mean": float(np.mean(f_steps)),
                             "converged": int(sum(f_conv)), "nonfinite": int(sum(1 for rc in f_rc if rc != 0))},
        "speedup_wall": t_fp64 / t_batch,
        "batched_fp32_then_fp64": {"wall_s": t_promoted, "steps_mean": float(np.mean(p_steps)),
                                   "converged": int(sum(1 for v in p_by if v == 1)),
                                   "nonfinite": int(sum(1 for v in p_by if v < 0)),
                                   "not_converged": int(sum(1 for v in p_by if v == 0))},
        "speedup_wall_fp64_finish": t_fp64 / t_promoted,
        "droplets_both_fp64_finish": len(drops_p),
        "steady_observables_fp64_finish_vs_fp64_rel": agreement(p_obs, drops_p),
        "converged_both": len(both),
        "steps_mean_both": {"batched_fp32": float(np.mean([b_steps[k] for k in both])) if both else None,
                            "per_droplet_fp64": float(np.mean([f_steps[k] for k in both])) if both else None},
        "droplets_both": len(drops), "evaporated_both": len(both) - len(drops),
        "steady_observables_fp32_vs_fp64_rel": agree,
        "per_item": [{"side": its[k]["side"], "R": its[k]["R"], "order": its[k]["order"], "G": its[k]["G"],
                      "tau": its[k]["tau"], "batched_steps": int(b_steps[k]), "batched_by": int(b_by[k]),
                      "fp64_steps": f_steps[k], "fp64_rc": f_rc[k], "fp64_wall_s": f_wall[k],
                      "obs_fp32": {q: b_obs[k][q] for q in ("max_u", "mean_u", "dp", "rho_min", "rho_max")},
                      "fp64_finish_steps": int(p_steps[k]), "fp64_finish_by": int(p_by[k]),
                      "obs_fp64_finish": {q: p_obs[k][q] for q in ("max_u", "mean_u", "dp", "rho_min", "rho_max")},
                      "obs_fp64": {q: f_obs[k][q] for q in ("max_u", "mean_u", "dp", "rho_min", "rho_max")}}
                     for k in range(n_items)],
    }


def main(argv=None):
    ap = argparse.ArgumentParser(description="droplet sweep to steady state: batched FP32 vs per-droplet FP64")
    ap.add_argument("--items", type=int, default=64)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--max-steps", type=int, default=200000)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    res = run(a.items, a.tol, a.max_steps, log=lambda m: print(m, flush=True))
    summary = {k: v for k, v in res.items() if k != "per_item"}
    print(json.dumps(summary), flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(res, fh, indent=1)
    return res


if __name__ == "__main__":
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main()
