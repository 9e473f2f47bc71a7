"""The 3D droplet at its full size (D3Q19 MRT, E8 3D force, G = -5,
tau = 1, 128^3, R = 24) against the FP64 oracle's own run of it over the
configuration's 20,000 steps, stored by
tests/golden/make_droplet_128_d3q19.py (Sec. 2, 3).

FP64 state: the observables at every stored checkpoint (every 500 steps)
within 1e-9 relative (Laplace jump: 1e-9 of p_in), and the density and
velocity along the x line through the centre at 2,000 steps and at the end
within 1e-10 absolute.
FP32 state (default storage shift), at 2,000 steps: the |u| norms within
1e-3 relative, the Laplace jump within 1e-4, the density extremes within
1e-5 relative, and the density along the line within 1e-5 relative where
the oracle's profile changes by less than 1e-4 per node and within 3e-3
absolute everywhere (interface nodes follow the interface's round-off
shift).  At the end: the |u| norms within 1e-3 and the Laplace jump
within 1e-4."""
import json
import os

import numpy as np
import pytest

from paper_1906_11027_amd import Sim
from tests.gpu_helpers import say
from workload import droplet_rho

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "droplet_128_d3q19_oracle.json")) as _fh:
    GOLD = json.load(_fh)
OBS = ("max_u", "mean_u", "l2_u", "rho_in", "rho_out", "rho_min", "rho_max", "mass", "radius")


def _sim(prec):
    rho0 = droplet_rho(tuple(GOLD["shape"]), GOLD["R"], seed=GOLD["seed"])
    return Sim(rho0, "D3Q19", order=GOLD["order"], G=GOLD["G"], tau=GOLD["tau"], collision=GOLD["collision"],
               precision=prec, obs_every=GOLD["every"])


def _line(out):
    y, z = GOLD["line_y"], GOLD["line_z"]
    return out["rho"][:, y, z], out["u"][:, :, y, z]


def _early():
    """(step, rho line, u line) stored mid-run, or the end of a short run."""
    e = GOLD.get("early")
    if e:
        return e["step"], np.asarray(e["rho_line"]), np.asarray(e["u_line"])
    return GOLD["steps"], np.asarray(GOLD["rho_line"]), np.asarray(GOLD["u_line"])


def test_fp64_matches_oracle_run():
    say("case droplet 128^3 D3Q19 MRT E8 fp64, %d steps" % GOLD["steps"])
    sim = _sim("fp64")
    worst = 0.0
    e_step, e_rho, e_u = _early()
    lines = []
    for ref in GOLD["traj"]:
        sim.step(GOLD["every"])
        ob = sim.observe(fields=False)["obs"]
        assert ob["step"] == ref["step"]
        for k in OBS:
            e = abs(ob[k] - ref[k]) / abs(ref[k])
            worst = max(worst, e)
            assert e <= 1e-9, (ref["step"], k, ob[k], ref[k])
        assert abs(ob["dp"] - ref["dp"]) <= 1e-9 * abs(ref["p_in"])
        if ref["step"] in (e_step, GOLD["steps"]):
            rho, u = _line(sim.observe())
            r_ref, u_ref = (e_rho, e_u) if ref["step"] == e_step else (np.asarray(GOLD["rho_line"]),
                                                                          np.asarray(GOLD["u_line"]))
            lines.append((ref["step"], float(np.max(np.abs(rho - r_ref))), float(np.max(np.abs(u - u_ref)))))
    sim.close()
    say("3D fp64: worst observable rel err %.2e; centre lines %s" % (
        worst, " ".join("t=%d rho %.1e u %.1e" % ln for ln in lines)))
    assert lines and all(er <= 1e-10 and eu <= 1e-10 for _, er, eu in lines)


def _fp32_observables(ob, ref):
    return {k: abs(ob[k] - ref[k]) / abs(ref[k]) for k in ("max_u", "mean_u", "l2_u", "dp", "rho_min", "rho_max")}


def test_fp32_matches_oracle_run():
    say("case droplet 128^3 D3Q19 MRT E8 fp32, %d steps" % GOLD["steps"])
    sim = _sim("fp32")
    e_step, r, _ = _early()
    sim.step(e_step)
    out = sim.observe()
    shift = sim.rho_ref
    ref = next(t for t in GOLD["traj"] if t["step"] == e_step)
    rel = _fp32_observables(out["obs"], ref)
    rho, _ = _line(out)
    bulk = 0.5 * np.abs(np.roll(r, -1) - np.roll(r, 1)) < 1e-4
    d = np.abs(rho - r)
    bulk_rel, any_abs = float(np.max(d[bulk] / r[bulk])), float(np.max(d))
    say("3D fp32 (shift %.4f) at %d steps: %s; line bulk rel %.1e, any abs %.1e" % (
        shift, e_step, " ".join("%s %.1e" % kv for kv in rel.items()), bulk_rel, any_abs))
    for k in ("max_u", "mean_u", "l2_u"):
        assert rel[k] <= 1e-3, (k, rel[k])
    assert rel["dp"] <= 1e-4
    assert rel["rho_min"] <= 1e-5 and rel["rho_max"] <= 1e-5
    assert bulk.sum() > r.size // 2
    assert bulk_rel <= 1e-5 and any_abs <= 3e-3
    if GOLD["steps"] > e_step:
        sim.step(GOLD["steps"] - e_step)
        rel = _fp32_observables(sim.observe(fields=False)["obs"], GOLD["traj"][-1])
        say("3D fp32 at %d steps: %s" % (GOLD["steps"], " ".join("%s %.1e" % kv for kv in rel.items())))
        for k in ("max_u", "mean_u", "l2_u"):
            assert rel[k] <= 1e-3, (k, rel[k])
        assert rel["dp"] <= 1e-4
    sim.close()
