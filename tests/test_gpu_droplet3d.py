"""The 3D droplet at its full size (D3Q19 MRT, E8 3D force, G = -5,
tau = 1, 128^3, R = 24) against the FP64 oracle's own 2,000-step run of
it, stored by tests/golden/make_droplet_128_d3q19.py (Sec. 2, 3).

FP64 state: the observables at every stored checkpoint within 1e-9
relative (Laplace jump: 1e-9 of p_in), and the final density and velocity
along the x line through the centre within 1e-10 absolute.
FP32 state (default storage shift): at the end, the |u| norms within 1e-3
relative, the Laplace jump within 1e-4, the density extremes within 1e-5
relative, and the density along the line within 1e-5 relative where the
oracle's profile changes by less than 1e-4 per node and within 3e-3
absolute everywhere (interface nodes follow the interface's round-off
shift)."""
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


def test_fp64_matches_oracle_run():
    say("case droplet 128^3 D3Q19 MRT E8 fp64, %d steps" % GOLD["steps"])
    sim = _sim("fp64")
    worst = 0.0
    for ref in GOLD["traj"]:
        sim.step(GOLD["every"])
        ob = sim.observe(fields=False)["obs"]
        assert ob["step"] == ref["step"]
        for k in OBS:
            e = abs(ob[k] - ref[k]) / abs(ref[k])
            worst = max(worst, e)
            assert e <= 1e-9, (ref["step"], k, ob[k], ref[k])
        assert abs(ob["dp"] - ref["dp"]) <= 1e-9 * abs(ref["p_in"])
    rho, u = _line(sim.observe())
    sim.close()
    er = float(np.max(np.abs(rho - np.asarray(GOLD["rho_line"]))))
    eu = float(np.max(np.abs(u - np.asarray(GOLD["u_line"]))))
    say("3D fp64: worst observable rel err %.2e; centre line rho %.1e u %.1e" % (worst, er, eu))
    assert er <= 1e-10 and eu <= 1e-10


def test_fp32_matches_oracle_run():
    say("case droplet 128^3 D3Q19 MRT E8 fp32, %d steps" % GOLD["steps"])
    sim = _sim("fp32")
    sim.step(GOLD["steps"])
    out = sim.observe()
    shift = sim.rho_ref
    sim.close()
    ob, ref = out["obs"], GOLD["traj"][-1]
    rel = {k: abs(ob[k] - ref[k]) / abs(ref[k]) for k in ("max_u", "mean_u", "l2_u", "dp", "rho_min", "rho_max")}
    rho, _ = _line(out)
    r = np.asarray(GOLD["rho_line"])
    bulk = 0.5 * np.abs(np.roll(r, -1) - np.roll(r, 1)) < 1e-4
    d = np.abs(rho - r)
    bulk_rel, any_abs = float(np.max(d[bulk] / r[bulk])), float(np.max(d))
    say("3D fp32 (shift %.4f): %s; line bulk rel %.1e, any abs %.1e" % (
        shift, " ".join("%s %.1e" % kv for kv in rel.items()), bulk_rel, any_abs))
    for k in ("max_u", "mean_u", "l2_u"):
        assert rel[k] <= 1e-3, (k, rel[k])
    assert rel["dp"] <= 1e-4
    assert rel["rho_min"] <= 1e-5 and rel["rho_max"] <= 1e-5
    assert bulk.sum() > r.size // 2
    assert bulk_rel <= 1e-5 and any_abs <= 3e-3
