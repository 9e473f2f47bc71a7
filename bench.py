#!/usr/bin/env python3
"""Throughput of the fused Shan-Chen step on one MI355X.

Headline workload: D2Q9 SRT, 256 x 256 periodic, E8 force stencil (24
neighbours), G = -5, tau = 1, psi = 1 - exp(-rho), droplet R = 40 (tanh
profile rho_l = 2.0 / rho_v = 0.15, width 2, jitter 1e-3 seed 2), state in
FP32 stored as f - w.  One "step" is one fused pass of psi(rho), the
interaction force, Guo-forced collision and pull streaming over the grid;
MLUPS = nodes x steps / time, with the state resident in HBM.

Also reported (same JSON line, key "extra"): the 128^3 D3Q19 MRT E8 droplet,
the HBM-bound grids 8192^2 (D2Q9 E8) and 320^3 (D3Q19 MRT E8), the larger
lattices of Sec. 3 at 8192^2 (D2Q13 E6 and D2Q25 E8 with the Peng-Robinson
psi and the exact difference method), the wall time of a 64^2 E4 droplet run
to its steady state and the batched 64-droplet sweep.

Timing: HIP events on the library's stream around K graph-replayed steps,
bracketed by device synchronisation.  The roofline takes the fused kernel's
time per launch as steps per launch (1, or 2 for the shapes that block
two steps in time) x the event-timed time per step, which includes the gap
between launches; its traffic is the tuned shape's measured HBM bytes per
launch (TRAFFIC_RATIO).  "frac" prices the algorithmic bytes (Q values read
and written per update) against 8 TB/s; "frac_counted" prices the bytes
the counters measured, so a two-step launch that moves half its
algorithmic bytes shows half the fraction there.  The CPU baseline is the
FP64 oracle on the host cores, on a bounded number of steps of the same
workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extra] [--no-cpu] [--no-steady]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS per GPU (D2Q9/D3Q19, E8 force) + wall-time to steady droplet"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "d2q9_e8_256": dict(lattice="D2Q9", shape=(256, 256), order=8, R=40, seed=2, collision="srt",
                        desc="D2Q9 SRT 256x256 periodic, E8 force (24 nbrs), G=-5, tau=1, "
                             "psi=1-exp(-rho), droplet R=40, FP32 shifted f-w"),
    "d3q19_mrt_e8_128": dict(lattice="D3Q19", shape=(128, 128, 128), order=8, R=24, seed=3,
                             collision="mrt",
                             desc="D3Q19 MRT 128^3 periodic, E8 3D force (92 nbrs), G=-5, tau=1, "
                                  "droplet R=24, FP32 shifted"),
    "d2q9_e8_8192": dict(lattice="D2Q9", shape=(8192, 8192), order=8, R=1600, seed=7, collision="srt",
                         desc="D2Q9 SRT 8192^2, E8, droplet R=1600, FP32 (HBM-bound size)"),
    "d3q19_mrt_e8_320": dict(lattice="D3Q19", shape=(320, 320, 320), order=8, R=64, seed=8,
                             collision="mrt",
                             desc="D3Q19 MRT 320^3, E8, droplet R=64, FP32 (HBM-bound size)"),
    # the larger lattices of Sec. 3 in the paper's own set-up: Peng-Robinson
    # psi at T/Tc = 0.85, exact difference method, droplet at the Maxwell
    # densities, at an HBM-bound size
    "d2q13_e6_pr_edm_8192": dict(lattice="D2Q13", shape=(8192, 8192), order=6, R=1600, seed=9, collision="srt",
                                 pr=0.85, forcing="edm", tau=11.0 / 12.0,
                                 desc="D2Q13 SRT 8192^2, E6, P-R psi T/Tc=0.85, EDM, tau=11/12, droplet "
                                      "R=1600, FP32"),
    "d2q25_e8_pr_edm_8192": dict(lattice="D2Q25", shape=(8192, 8192), order=8, R=1600, seed=10, collision="srt",
                                 pr=0.85, forcing="edm", tau=19.0 / 24.0,
                                 desc="D2Q25 SRT 8192^2, E8, P-R psi T/Tc=0.85, EDM, tau=19/24, droplet "
                                      "R=1600, FP32"),
    # the FP64 state at the HBM-bound sizes (same droplets)
    "d2q9_e8_8192_fp64": dict(lattice="D2Q9", shape=(8192, 8192), order=8, R=1600, seed=7, collision="srt",
                              precision="fp64", desc="D2Q9 SRT 8192^2, E8, droplet R=1600, FP64 state"),
    "d3q19_mrt_e8_320_fp64": dict(lattice="D3Q19", shape=(320, 320, 320), order=8, R=64, seed=8,
                                  collision="mrt", precision="fp64",
                                  desc="D3Q19 MRT 320^3, E8, droplet R=64, FP64 state"),
}
Q_OF = {"D2Q9": 9, "D3Q19": 19, "D2Q13": 13, "D2Q25": 25}

# HBM traffic per launch relative to the algorithmic bytes of the launch
# (steps per launch x read Q + write Q per node), (fetch, write), from
# rocprofv3 FETCH_SIZE / WRITE_SIZE runs of this script (one counter per run) scaled
# by what the same counters read for a 256 MiB device copy (the counter
# summary under profiles/).  Keyed by workload and launch shape; a shape
# without an entry reports traffic null.  Re-measure after a kernel change.
TRAFFIC_RATIO = {
    # measured with the kernels of this tree (pair-increment collisions,
    # unwrapped pulls for interior two-step tiles; the D3Q19 FP32 window
    # marches re-counted after the state accesses took the global address
    # space, which changed their register allocation; the any-lattice and
    # the single-grid D2Q9 two-step shapes and the FP64 D3Q19 marches
    # re-counted with their non-temporal stores)
    ("d2q9_e8_256", "tile2x32x8t1024"): (0.678, 0.500),
    ("d2q9_e8_256", "tile2x32x8t512"): (0.685, 0.500),
    ("d2q9_e8_256", "tile2x16x16"): (0.907, 0.557),
    ("d2q9_e8_256", "tile2x32x16"): (0.691, 0.500),
    ("d2q9_e8_256", "tile2x32x32"): (0.684, 0.500),
    ("d2q9_e8_256", "tile2x32x8"): (0.697, 0.500),
    ("d2q9_e8_256", "tile2x64x16"): (0.687, 0.500),
    ("d2q9_e8_256", "tile2x64x8"): (0.695, 0.500),
    ("d2q9_e8_256", "tile32x8r1"): (1.157, 1.000),
    ("d2q9_e8_256", "tile64x4r1"): (1.159, 1.000),
    ("d2q9_e8_8192", "tile2x32x8t1024"): (0.626, 0.500),
    ("d2q9_e8_8192", "tile2x32x8t512"): (0.626, 0.500),
    ("d2q9_e8_8192", "tile2x16x16"): (1.257, 0.517),
    ("d2q9_e8_8192", "tile2x32x16"): (0.633, 0.500),
    ("d2q9_e8_8192", "tile2x32x32"): (0.630, 0.500),
    ("d2q9_e8_8192", "tile2x32x8"): (0.627, 0.500),
    ("d2q9_e8_8192", "tile2x64x16"): (0.563, 0.500),
    ("d2q9_e8_8192", "tile2x64x8"): (0.563, 0.500),
    ("d2q9_e8_8192", "tile64x16r4"): (1.543, 1.000),
    ("d3q19_mrt_e8_320", "march64x8r1h64pf1"): (1.431, 1.000),
    ("d3q19_mrt_e8_320", "march64x8r1h32pf1"): (1.568, 1.000),
    ("d3q19_mrt_e8_320", "march64x12r1h64pf1"): (1.322, 1.000),
    ("d3q19_mrt_e8_320", "march64x12r1h32pf1"): (1.395, 1.000),
    ("d3q19_mrt_e8_320", "march64x12r1h16pf1"): (1.523, 1.000),
    ("d3q19_mrt_e8_320", "rl64x8h64w4"): (2.726, 1.000),
    ("d3q19_mrt_e8_320", "rl64x8h32w4"): (2.818, 1.000),
    # the three persistent 64 x 8 shapes share one grid (one block per CU):
    # their mean over the autotuner's dispatches
    ("d3q19_mrt_e8_320", "pmarch64x8r1h64pf1"): (1.331, 1.000),
    ("d3q19_mrt_e8_320", "pmarch64x8r1h32pf1"): (1.331, 1.000),
    ("d3q19_mrt_e8_320", "pmarch64x8r1h16pf1"): (1.331, 1.000),
    ("d3q19_mrt_e8_128", "march64x8r1h16pf1"): (1.253, 1.000),
    ("d3q19_mrt_e8_128", "march64x8r1h32pf1"): (1.198, 1.000),
    ("d3q19_mrt_e8_128", "march64x8r1h64pf1"): (1.198, 1.000),
    ("d3q19_mrt_e8_128", "march64x8r1h16"): (1.253, 1.000),
    ("d3q19_mrt_e8_128", "pmarch64x8r1h16pf1"): (1.253, 1.000),
    ("d3q19_mrt_e8_128", "pmarch64x8r1h32pf1"): (1.198, 1.000),
    ("d3q19_mrt_e8_128", "pmarch64x8r1h64pf1"): (1.198, 1.000),
    ("d3q19_mrt_e8_128", "rl64x8h64w4"): (1.196, 1.000),
    ("d3q19_mrt_e8_128", "rl64x8h32w4"): (1.265, 1.000),
    # two-step any-lattice shapes: re-counted with the windowed LDS copy
    ("d2q13_e6_pr_edm_8192", "wide2x32x8t256"): (0.628, 0.500),
    ("d2q13_e6_pr_edm_8192", "wide2x64x8t512"): (0.564, 0.500),
    ("d2q13_e6_pr_edm_8192", "wide2x64x16t1024"): (0.564, 0.500),
    ("d2q13_e6_pr_edm_8192", "wide2x128x8t1024"): (0.534, 0.500),
    ("d2q13_e6_pr_edm_8192", "wide2x64x8t1024"): (0.563, 0.500),
    ("d2q13_e6_pr_edm_8192", "wide2x64x12t768"): (0.564, 0.500),
    ("d2q13_e6_pr_edm_8192", "wide2x64x12t1024"): (0.564, 0.500),
    ("d2q13_e6_pr_edm_8192", "wide2x64x16t768"): (0.565, 0.500),
    ("d2q13_e6_pr_edm_8192", "wide2x128x12t1024"): (0.549, 0.500),
    ("d2q13_e6_pr_edm_8192", "wide128x16r2"): (1.360, 1.000),
    ("d2q13_e6_pr_edm_8192", "wide256x8r2"): (1.355, 1.000),
    ("d2q13_e6_pr_edm_8192", "wide64x16r2"): (1.795, 1.000),
    ("d2q13_e6_pr_edm_8192", "wide64x16r4"): (1.863, 1.000),
    # D2Q25 E8 128 x 8 and 128 x 12 do not fit in LDS and run the 32 x 8 tile
    ("d2q25_e8_pr_edm_8192", "wide2x32x8t256"): (0.677, 0.500),
    ("d2q25_e8_pr_edm_8192", "wide2x128x8t1024"): (0.677, 0.500),
    ("d2q25_e8_pr_edm_8192", "wide2x128x12t1024"): (0.677, 0.500),
    ("d2q25_e8_pr_edm_8192", "wide2x64x8t512"): (0.581, 0.500),
    ("d2q25_e8_pr_edm_8192", "wide2x64x8t1024"): (0.609, 0.500),
    ("d2q25_e8_pr_edm_8192", "wide2x64x12t768"): (0.600, 0.500),
    ("d2q25_e8_pr_edm_8192", "wide2x64x12t1024"): (0.597, 0.500),
    ("d2q25_e8_pr_edm_8192", "wide2x64x16t1024"): (0.608, 0.500),
    ("d2q25_e8_pr_edm_8192", "wide2x64x16t768"): (0.617, 0.500),
    ("d2q25_e8_pr_edm_8192", "wide128x16r2"): (1.442, 1.000),
    ("d2q25_e8_pr_edm_8192", "wide256x8r2"): (1.407, 1.000),
    ("d2q25_e8_pr_edm_8192", "wide64x16r2"): (1.796, 1.000),
    ("d2q25_e8_pr_edm_8192", "wide64x16r4"): (2.138, 1.000),
    # FP64 state (write above 1: the shapes whose window spills to scratch)
    ("d2q9_e8_8192_fp64", "tile2x16x16"): (0.626, 0.500),
    ("d2q9_e8_8192_fp64", "tile2x32x8"): (0.563, 0.500),
    ("d2q9_e8_8192_fp64", "tile2x32x8t512"): (0.563, 0.500),
    ("d2q9_e8_8192_fp64", "tile2x32x8t1024"): (0.563, 0.500),
    ("d2q9_e8_8192_fp64", "tile2x32x16"): (0.563, 0.500),
    ("d2q9_e8_8192_fp64", "tile2x32x32"): (0.565, 0.500),
    ("d2q9_e8_8192_fp64", "tile2x64x8"): (0.532, 0.500),
    ("d2q9_e8_8192_fp64", "tile2x64x16"): (0.532, 0.500),
    ("d3q19_mrt_e8_320_fp64", "march32x16h16"): (1.646, 1.000),
    ("d3q19_mrt_e8_320_fp64", "march32x16h32"): (1.369, 1.000),
    ("d3q19_mrt_e8_320_fp64", "march32x8r1h32pf1"): (1.436, 1.000),
    ("d3q19_mrt_e8_320_fp64", "march32x8r1h64pf1"): (1.321, 1.000),
    ("d3q19_mrt_e8_320_fp64", "pmarch64x8r1h64pf1"): (3.165, 1.902),
    ("d3q19_mrt_e8_320_fp64", "pmarch64x8r1h32pf1"): (3.165, 1.902),
    ("d3q19_mrt_e8_320_fp64", "pmarch64x8r1h16pf1"): (3.165, 1.902),
    # the persistent 32 x 8 shapes share one grid: their mean
    ("d3q19_mrt_e8_320_fp64", "pmarch32x8r1h64pf1"): (1.341, 1.000),
    ("d3q19_mrt_e8_320_fp64", "pmarch32x8r1h32pf1"): (1.341, 1.000),
    ("d3q19_mrt_e8_320_fp64", "rl64x8h64w4"): (2.345, 1.000),
    ("d3q19_mrt_e8_320_fp64", "rl64x8h32w4"): (2.460, 1.000),
}



def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bytes_per_node(lattice, precision="fp32"):
    # read Q + write Q values of the state (algorithmic traffic)
    return 2 * Q_OF[lattice] * (8 if precision == "fp64" else 4)


def sim_kwargs(w):
    """Library parameters of a workload (exp psi unless it names a P-R
    reduced temperature) and its initial density field."""
    from paper_1906_11027_amd import eos as P
    from workload import droplet_rho

    kw = dict(order=w["order"], collision=w["collision"], forcing=w.get("forcing", "guo"), tau=w.get("tau", 1.0))
    dens = {}
    if "pr" in w:
        e = P.params_at(w["pr"])
        rv, rl = P.maxwell(e)
        kw.update(psi="pr", eos=e, G=-1.0)
        dens = dict(rho_l=rl, rho_v=rv)
    rho0 = droplet_rho(w["shape"], w["R"], seed=w["seed"], **dens)
    return kw, rho0


def measure(name, steps, warmup, kernel_launches=50):
    import torch

    from paper_1906_11027_amd import Sim
    from paper_1906_11027_amd import sc_lbm as B

    w = WORKLOADS[name]
    kw, rho0 = sim_kwargs(w)
    # pick the launch shape by timing every candidate under graph replay
    # (cached for variant -1); small grids get more steps per timing run
    nodes = 1
    for d in w["shape"]:
        nodes *= int(d)
    prec = w.get("precision", "fp32")
    tuned = B.sc_lbm_autotune(B.make_params(w["lattice"], w["shape"], precision=prec, **kw),
                              steps=256 if nodes < 1 << 20 else 32)
    log("autotune %s: variant %d, %.4f ms/step" % (name, tuned[0], tuned[1]))
    stream = torch.cuda.Stream()
    sim = Sim(rho0, w["lattice"], precision=prec, stream=stream, **kw)
    assert sim.stream == stream.cuda_stream, "library is not on the timed stream"
    n = rho0.size
    del rho0
    sim.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    # the device cannot finish before the host has enqueued the work it times
    # only if the events bracket it: cross-check against the wall clock
    if ms < 0.5 * wall * 1e3 and wall > 0.05:
        raise RuntimeError("event time %.3f ms << wall %.3f ms: events do not bracket the steps"
                           % (ms, wall * 1e3))
    # per-launch kernel duration: events around single (non-graph) launches
    ea = [torch.cuda.Event(enable_timing=True) for _ in range(kernel_launches)]
    eb = [torch.cuda.Event(enable_timing=True) for _ in range(kernel_launches)]
    for k in range(kernel_launches):
        ea[k].record(stream)
        sim.step(1)
        eb[k].record(stream)
    torch.cuda.synchronize()
    kms = sorted(a.elapsed_time(b) for a, b in zip(ea, eb))
    kmean = sum(kms) / len(kms)
    ob = sim.observe(fields=False)["obs"]
    variant = sim.variant
    sim_spl = sim.steps_per_launch
    sim.close()
    ok = ob["nonfinite"] == 0 and ob["mass"] > 0
    mlups = n * steps / (ms * 1e-3) / 1e6
    bpn = bytes_per_node(w["lattice"], prec)
    # one fused launch per step: its average duration is the graph-timed
    # per-step time (an upper bound: it includes the gap between launches)
    achieved = bpn * n / (ms / steps * 1e-3) / 1e9
    spl = sim_spl
    tr = TRAFFIC_RATIO.get((name, variant))
    traffic = None if tr is None else (tr[0] + tr[1]) * spl * bpn * n / 2.0
    return {
        "workload": name, "desc": w["desc"], "nodes": n, "steps": steps, "ms_total": ms,
        "ms_per_step": ms / steps, "wall_s": wall, "mlups": mlups,
        "single_launch_ms_mean": kmean, "single_launch_ms_median": kms[len(kms) // 2],
        "bytes_per_node": bpn,
        "achieved_gbs": achieved, "frac": achieved / HBM_PEAK_GBS, "variant": variant,
        "finite": bool(ok), "max_u": ob["max_u"], "traffic_bytes": traffic,
        "traffic_ratio": None if tr is None else (tr[0] + tr[1]) / 2.0,
        # the same time against the bytes the counters measured for this
        # shape: the share of 8 TB/s the kernel really moves
        "frac_counted": None if tr is None else achieved * (tr[0] + tr[1]) / 2.0 / HBM_PEAK_GBS,
        "steps_per_launch": spl, "launch_ms": spl * ms / steps, "bytes_per_launch": spl * bpn * n,
    }


def copy_ceiling(nbytes=1 << 30, reps=8):
    """Streaming ceiling of the GPU: a device-to-device copy of 1 GiB timed
    with events (read + write bytes per second, best of `reps`)."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = 1e30
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    return {"bytes": 2 * nbytes, "ms": best, "gbs": 2 * nbytes / (best * 1e-3) / 1e9}


def steady_droplet(shape=(64, 64), R=16, seed=1, order=4, precision="fp32", max_steps=400000):
    """A droplet run to steady state on the GPU (default: the 64^2 E4 droplet,
    R = 16)."""
    import torch

    from paper_1906_11027_amd import Sim
    from workload import droplet_rho

    rho0 = droplet_rho(shape, R, seed=seed)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim = Sim(rho0, "D2Q9", order=order, stream=stream, obs_every=100, precision=precision)
    rc, done = sim.step(max_steps, tol=1e-10)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ob = sim.observe(fields=False)["obs"]
    sim.close()
    rule = ("FP32: on 3 consecutive checks, or max|u| of 50 checks on a line within the state's resolution "
            "that stays in it for 300 more checks"
            if precision == "fp32" else "FP64: the literal rule")
    return {"workload": "D2Q9 SRT %dx%d E%d droplet R=%d, %s, to max|u| change < 1e-10 per 100 steps (%s)"
                        % (shape[0], shape[1], order, R, precision.upper(), rule),
            "steps": done, "wall_s": wall, "max_u": ob["max_u"], "dp": ob["dp"], "rc": rc,
            "converged_by": ob["converged_by"]}


def _sweep_items():
    from workload import droplet_rho, sweep_items
    its = sweep_items(64, seed=1906)
    return its, [{"rho0": droplet_rho((it["side"],) * 2, it["R"], seed=it["seed"]), "order": it["order"],
                  "G": it["G"], "tau": it["tau"]} for it in its]


def batched_sweep(steps=200):
    """64 droplets drawn like the sweep configuration (sides 64..512, R, G,
    tau, stencil order per item) advanced together: the batched shape tuner's
    choice, then every batched launch shape."""
    import torch

    from paper_1906_11027_amd import Batch, batch_autotune
    from paper_1906_11027_amd import sc_lbm as B

    _, items = _sweep_items()
    nodes = sum(it["rho0"].size for it in items)
    tuned, tuned_ms = batch_autotune(items, steps=64)
    log("batch autotune: variant %d, %.4f ms/step" % (tuned, tuned_ms))
    st = torch.cuda.Stream()
    shapes = {}
    auto = None
    for v in [tuned] + list(range(B.lib().sc_lbm_batch_num_variants())):
        bt = Batch(items, stream=st, variant=v)
        name = bt.variant
        bt.step(20)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        bt.step(steps)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        bt.close()
        if auto is None:
            auto = (name, ms)
        else:
            shapes[name] = round(nodes / ms / 1e3, 1)
    name, ms = auto
    return {"workload": "64 D2Q9 droplets, sides U{64..512}, R, G, tau, order per item (PCG64 seed 1906), "
                        "FP32, %d steps" % steps, "nodes": nodes, "variant": name, "tuned_variant": tuned,
            "ms_per_step": ms,
            "mlups": nodes / ms / 1e3, "achieved_gbs": nodes * 72 / ms / 1e6, "mlups_by_variant": shapes}


def sweep_steady(max_steps=200000, tol=1e-10, variant=-1):
    """Wall time for the 64 sweep droplets to reach a steady state (max |u|
    changing by less than tol between checks 100 steps apart): one batched
    FP32 run with its resolution rules, then finished in FP64 to the literal
    rule (sc_lbm_batch_promote), against plain per-droplet FP64 runs one
    after the other.  Both include creation and every check."""
    import numpy as np
    import torch

    from paper_1906_11027_amd import Batch, Sim

    its, items = _sweep_items()
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt = Batch(items, stream=st, obs_every=100, variant=variant)
    bt.step(max_steps, tol=tol)
    torch.cuda.synchronize()
    t32 = time.perf_counter() - t0
    s32 = [bt.status(k) for k in range(len(items))]
    bt.promote()
    bt.step(max_steps, tol=tol)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    sb = [bt.status(k) for k in range(len(items))]
    ob = [bt.observe(k, fields=False)["obs"] for k in range(len(items))]
    bt.close()
    t0 = time.perf_counter()
    s64, o64 = [], []
    for it in items:
        sim = Sim(it["rho0"], "D2Q9", order=it["order"], G=it["G"], tau=it["tau"], precision="fp64",
                  obs_every=100, stream=st)
        rc, done = sim.step(max_steps, tol=tol)
        s64.append((int(done), sim.observe(fields=False)["obs"]["converged_by"] if rc == 0 else -1))
        o64.append(sim.observe(fields=False)["obs"])
        sim.close()
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    both = [k for k in range(len(items)) if sb[k][1] == 1 and s64[k][1] == 1
            and o64[k]["rho_max"] - o64[k]["rho_min"] > 0.5]
    rel = [abs(ob[k]["max_u"] - o64[k]["max_u"]) / o64[k]["max_u"] for k in both]
    return {"workload": "64 sweep droplets to max|u| change < %g per 100 steps: batched FP32 (its rules) then "
                        "FP64 (literal rule) vs one-by-one FP64 (literal rule), %d steps at most per stage"
                        % (tol, max_steps),
            "batched_fp32_s": t32, "batched_fp32_then_fp64_s": t_batch, "per_droplet_fp64_s": t64,
            "speedup": t64 / t_batch,
            "converged_batched": sum(1 for s in sb if s[1] == 1),
            "converged_per_droplet": sum(1 for s in s64 if s[1] == 1),
            "quarantined": sum(1 for s in sb if s[1] == -1),
            "steady_max_u_rel_diff_median": float(np.median(rel)) if rel else None,
            "steady_max_u_rel_diff_max": float(np.max(rel)) if rel else None}


def cpu_baseline(name, target_s=15.0):
    from oracle import oracle as O
    from workload import droplet_rho

    w = WORKLOADS[name]
    rho0 = droplet_rho(w["shape"], w["R"], seed=w["seed"])
    o = O.Oracle(rho0, w["lattice"], order=w["order"], collision=w["collision"])
    t0 = time.perf_counter()
    o.step(2)
    dt = (time.perf_counter() - t0) / 2
    k = max(2, int(target_s / max(dt, 1e-6)))
    t0 = time.perf_counter()
    o.step(k)
    el = time.perf_counter() - t0
    return {"value": rho0.size * k / el / 1e6, "unit": "MLUPS", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": "%d steps of the %s workload (FP64 oracle, OpenMP over rows)" % (k, name)}


def kernel_label(w, r):
    """The fused step kernel a workload's tuned shape runs."""
    t = "double" if w.get("precision") == "fp64" else "float"
    if w["lattice"] == "D2Q9":
        k = "k_d2q9_tile2" if r["steps_per_launch"] == 2 else "k_d2q9_tile"
        return "%s<%s, %d, ...> (%s)" % (k, t, w["order"], r["variant"])
    if w["lattice"] == "D3Q19":
        return "k_d3q19_march<%s, %d, %s, ...> (%s)" % (t, w["order"], str(w["collision"] == "mrt").lower(),
                                                        r["variant"])
    return "k_wide_tile<%s, %s, %d, ...> (%s)" % (t, w["lattice"], w["order"], r["variant"])


def cpu_one_core(name, target_s=8.0):
    """The same oracle timing with one OpenMP thread, in a child process (the
    thread count is fixed when the oracle library loads)."""
    import subprocess
    code = "import json, bench; print(json.dumps(bench.cpu_baseline(%r, %r)))" % (name, target_s)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], cwd=os.path.dirname(os.path.abspath(__file__)), env=env,
                       capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        return {"error": r.stderr.strip().splitlines()[-1] if r.stderr.strip() else "rc %d" % r.returncode}
    return json.loads(r.stdout.strip().splitlines()[-1])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="d2q9_e8_256", choices=sorted(WORKLOADS))
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-steady", action="store_true",
                    help="skip the runs to steady state (for kernel traces: they launch ~10^6 kernels)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run 5 device copies of 256 MiB (reference dispatches for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(a domain would shard into slabs along its slowest axis with a halo exchange per step; "
              "not built)", file=sys.stderr)
        sys.exit(2)

    # before the GPU is touched: the one-core oracle timing runs in a child
    one_core = None
    if not args.no_cpu:
        one_core = cpu_one_core(args.workload)
        log("cpu one core:", json.dumps(one_core))

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.copy_calibration:
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    main_r = measure(args.workload, args.steps, args.warmup)
    log("main:", json.dumps(main_r))
    extra = {}
    if not args.no_extra:
        for name, st in (("d3q19_mrt_e8_128", 200), ("d2q9_e8_8192", 100), ("d3q19_mrt_e8_320", 40),
                         ("d2q13_e6_pr_edm_8192", 40), ("d2q25_e8_pr_edm_8192", 30),
                         ("d2q9_e8_8192_fp64", 40), ("d3q19_mrt_e8_320_fp64", 20)):
            if name == args.workload:
                continue
            r = measure(name, st, 10, kernel_launches=10)
            log(name + ":", json.dumps(r))
            extra[name] = {k: r[k] for k in ("mlups", "ms_per_step", "single_launch_ms_mean",
                                             "achieved_gbs", "frac", "frac_counted", "variant", "finite",
                                             "traffic_ratio", "steps_per_launch")}
        cc = copy_ceiling()
        log("copy:", json.dumps(cc))
        extra["copy_ceiling"] = cc
        # counted traffic against what a device copy streams on this GPU
        for r in extra.values():
            if isinstance(r, dict) and r.get("traffic_ratio"):
                r["frac_of_copy"] = r["achieved_gbs"] * r["traffic_ratio"] / cc["gbs"]
        if not args.no_steady:
            sd = steady_droplet()
            log("steady:", json.dumps(sd))
            extra["steady_droplet"] = sd
            # the headline droplet (256^2, E8, R = 40) to steady state, both states
            for prec in ("fp32", "fp64"):
                sd = steady_droplet((256, 256), 40, 2, 8, prec)
                log("steady 256 %s:" % prec, json.dumps(sd))
                extra["steady_droplet_256_e8_" + prec] = sd
        bs = batched_sweep()
        log("batch:", json.dumps(bs))
        extra["batched_sweep_64"] = bs
        if not args.no_steady:
            ss = sweep_steady(variant=bs["tuned_variant"])
            log("sweep steady:", json.dumps(ss))
            extra["sweep_steady_64"] = ss
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(args.workload)
        log("cpu:", json.dumps(cpu))

    w = WORKLOADS[args.workload]
    line = {
        "metric": METRIC,
        "value": round(main_r["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w.get("precision", "fp32"),
        "data": "synthetic",
        "config": {"workload": w["desc"], "nodes": main_r["nodes"], "lattice": w["lattice"],
                   "grid": list(w["shape"]), "stencil_order": w["order"], "variant": main_r["variant"]},
        # the 256^2 state (2 x 2.4 MB) stays in the caches: the two-step launch
        # is bound by latency (loads, LDS, barriers), not by HBM bandwidth;
        # it is still priced against the HBM peak, and the HBM-bound sizes of
        # the same kernels are under "extra"
        "roofline": {"bound": "latency", "achieved": round(main_r["achieved_gbs"], 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(main_r["frac"], 4),
                     "traffic": main_r["traffic_bytes"],
                     "traffic_ratio": main_r["traffic_ratio"],
                     "frac_counted": None if main_r["frac_counted"] is None else round(main_r["frac_counted"], 4),
                     "kernel": kernel_label(w, main_r),
                     "steps_per_launch": main_r["steps_per_launch"],
                     "kernel_ms_mean": main_r["launch_ms"],
                     "bytes_per_launch": main_r["bytes_per_launch"]},
        "cpu_baseline": cpu,
        "extra": dict(extra, cpu_oracle_one_core=one_core) if one_core else extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
